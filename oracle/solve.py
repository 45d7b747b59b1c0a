"""Applying the spaQR factor and CGLS (oracle, test infrastructure only).

The factorization gives Q^T (A D^-1) W^-1 ~ I (Section 2.7) with W a product
of sparse triangular and orthogonal factors that is never formed: W^-1 and
W^-T are applied op by op (Section 1: W is kept as a sequence of Householder
vectors and triangular factors).  The preconditioned solver is CGLS on
A D^-1 W^-1 (Section 4), stopped on the normal-equation residual.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from . import dense


def apply_winv(ops, y):
    """x = W^-1 y, ops traversed last to first."""
    x = np.array(y, dtype=np.float64, copy=True)
    for op in reversed(ops):
        kind = op[0]
        if kind == "elim":
            _, s, nb, R = op
            cs = s.shape[0]
            t = x[s] - R[:, cs:] @ x[nb] if nb.shape[0] else x[s]
            x[s] = sl.solve_triangular(R[:, :cs], t, lower=False)
        elif kind == "scale":
            _, p, R = op
            x[p] = sl.solve_triangular(R, x[p], lower=False)
        else:
            _, p, V, tau = op
            x[p] = dense.apply_q(V, tau, x[p])
    return x


def apply_winvt(ops, y):
    """x = W^-T y, ops traversed first to last with transposes."""
    x = np.array(y, dtype=np.float64, copy=True)
    for op in ops:
        kind = op[0]
        if kind == "elim":
            _, s, nb, R = op
            cs = s.shape[0]
            xs = sl.solve_triangular(R[:, :cs], x[s], trans="T", lower=False)
            x[s] = xs
            if nb.shape[0]:
                x[nb] -= R[:, cs:].T @ xs
        elif kind == "scale":
            _, p, R = op
            x[p] = sl.solve_triangular(R, x[p], trans="T", lower=False)
        else:
            _, p, V, tau = op
            x[p] = dense.apply_qt(V, tau, x[p])
    return x


def csr_matvec(row_ptr, col_idx, vals, v, M):
    out = np.zeros(M)
    rows = np.repeat(np.arange(M), np.diff(row_ptr))
    np.add.at(out, rows, vals * v[col_idx])
    return out


def csr_rmatvec(row_ptr, col_idx, vals, u, N):
    rows = np.repeat(np.arange(row_ptr.shape[0] - 1), np.diff(row_ptr))
    return np.bincount(col_idx, weights=vals * u[rows], minlength=N)


class Operator:
    """A (unscaled) as CSR, with the column norms D of the factorization."""

    def __init__(self, fac):
        an = fac.an
        self.fac = fac
        self.M, self.N = an.M, an.N
        self.row_ptr, self.col_idx, self.vals = an.row_ptr, an.col_idx, an.vals
        self.D = an.D

    def A(self, v):
        return csr_matvec(self.row_ptr, self.col_idx, self.vals, v, self.M)

    def At(self, u):
        return csr_rmatvec(self.row_ptr, self.col_idx, self.vals, u, self.N)

    def Mv(self, y):        # D^-1 W^-1 y
        return apply_winv(self.fac.ops, y) / self.D

    def Mtv(self, t):       # W^-T D^-1 t
        return apply_winvt(self.fac.ops, t / self.D)


def norm2_estimate(op: Operator, iters: int = 30) -> float:
    """||A||_2 from power iterations on A^T A, started from the all-ones vector."""
    v = np.ones(op.N)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = op.At(op.A(v))
        lam = np.linalg.norm(w)
        if lam == 0.0:
            return 0.0
        v = w / lam
    return float(np.sqrt(lam))


def cgls(op: Operator, b, tol=1e-10, max_iter=200, normA=None):
    """CGLS on (A D^-1 W^-1) y = b, x = D^-1 W^-1 y.

    Stops when ||A^T (b - A x)|| <= tol * ||A||_2 * ||b|| (the recursively
    updated residual is tested each iteration, the true one at exit).
    Returns (x, info).
    """
    if normA is None:
        normA = norm2_estimate(op)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    y = np.zeros(op.N)
    r = b.copy()
    t = op.At(r)
    s = op.Mtv(t)
    p = s.copy()
    gamma = float(s @ s)
    hist = [float(np.linalg.norm(t)) / (normA * nb)]
    it = 0
    while hist[-1] > tol and it < max_iter:
        q = op.A(op.Mv(p))
        alpha = gamma / float(q @ q)
        y += alpha * p
        r -= alpha * q
        t = op.At(r)
        it += 1
        hist.append(float(np.linalg.norm(t)) / (normA * nb))
        s = op.Mtv(t)
        gnew = float(s @ s)
        p = s + (gnew / gamma) * p
        gamma = gnew
    x = op.Mv(y)
    rt = b - op.A(x)
    true_res = float(np.linalg.norm(op.At(rt))) / (normA * nb)
    atb = float(np.linalg.norm(op.At(b)))
    paper_res = float(np.linalg.norm(op.At(rt))) / atb
    return x, dict(iters=it, history=hist, residual=true_res, paper_residual=paper_res, normA=normA,
                   converged=hist[-1] <= tol)


def csne(op: Operator, b):
    """One-shot seminormal solve x = D^-1 W^-1 W^-T D^-1 A^T b (Section 1)."""
    return op.Mv(op.Mtv(op.At(np.asarray(b, dtype=np.float64))))


def csne_refined(op: Operator, b, tol=1e-10, max_steps=50, normA=None):
    """Corrected seminormal equations with iterative refinement (Section 1).

    The factor gives A^T A ~ D W^T W D, so one seminormal solve is
    x = D^-1 W^-1 W^-T D^-1 A^T b.  Each refinement step solves the same
    system for the residual's normal-equation right-hand side and adds the
    correction:
        x_0     = M A^T b,
        x_{k+1} = x_k + M A^T (b - A x_k),   M = D^-1 W^-1 W^-T D^-1,
    until ||A^T (b - A x)|| <= tol ||A||_2 ||b|| (tested before every step)
    or max_steps corrections were added.  Returns (x, info) with info
    holding the number of corrections, the residual history and the final
    residual in both normalisations.
    """
    if normA is None:
        normA = norm2_estimate(op)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    x = op.Mv(op.Mtv(op.At(b)))
    hist = []
    steps = 0
    while True:
        r = b - op.A(x)
        t = op.At(r)
        hist.append(float(np.linalg.norm(t)) / (normA * nb))
        if hist[-1] <= tol or steps >= max_steps:
            break
        x = x + op.Mv(op.Mtv(t))
        steps += 1
    atb = float(np.linalg.norm(op.At(b)))
    return x, dict(steps=steps, history=hist, residual=hist[-1], paper_residual=hist[-1] * normA * nb / atb,
                   normA=normA, converged=hist[-1] <= tol)

