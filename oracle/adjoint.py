"""Gradients of the least-squares solution (oracle, test infrastructure only).

x*(A, b) = argmin ||A x - b||_2 for A of full column rank satisfies the
normal equations A^T A x = A^T b.  Differentiating them gives, for a loss
L(x) with g = dL/dx and the adjoint lambda solving A^T A lambda = g,

    dL/db      = A lambda
    dL/dA_ij   = r_i lambda_j - (A lambda)_i x_j,     r = b - A x,

restricted to the stored nonzeros of A.  ``grads_direct`` writes this
definition out with a sparse direct solve of the normal equations.
``adjoint_pcg`` reaches the same lambda the way the GPU path does: CG on
A^T A preconditioned by (W^T W)^-1 in the column-scaled variables, the
spaQR factor of A D^-1 being reused (Q^T A D^-1 W^-1 ~ I, Section 2.7, so
A^T A ~ D W^T W D).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import solve


def _csr(row_ptr, col_idx, vals, M, N):
    return sp.csr_matrix((vals, col_idx, row_ptr), shape=(M, N))


def lstsq_solution(row_ptr, col_idx, vals, b, M, N):
    """x* from the normal equations, sparse direct (A of full column rank)."""
    A = _csr(row_ptr, col_idx, vals, M, N)
    return spla.spsolve((A.T @ A).tocsc(), A.T @ b)


def grads_from_lambda(row_ptr, col_idx, vals, b, x, lam, M):
    """(dL/db, dL/dvals) for a given adjoint lambda."""
    rows = np.repeat(np.arange(M), np.diff(row_ptr))
    Ax = solve.csr_matvec(row_ptr, col_idx, vals, x, M)
    r = b - Ax
    Al = solve.csr_matvec(row_ptr, col_idx, vals, lam, M)
    g_vals = r[rows] * lam[col_idx] - Al[rows] * x[col_idx]
    return Al, g_vals


def grads_direct(row_ptr, col_idx, vals, b, x, g, M, N):
    """Gradients by the definition: lambda = (A^T A)^-1 g, sparse direct."""
    A = _csr(row_ptr, col_idx, vals, M, N)
    lam = spla.spsolve((A.T @ A).tocsc(), np.asarray(g, dtype=np.float64))
    gb, gv = grads_from_lambda(row_ptr, col_idx, vals, b, x, lam, M)
    return gb, gv, lam


def adjoint_pcg(op: solve.Operator, g, tol=1e-12, max_iter=500):
    """lambda with A^T A lambda = g by preconditioned CG.

    In scaled variables mu = D lambda the system is (Ahat^T Ahat) mu = D^-1 g
    with Ahat = A D^-1, preconditioned by W^-1 W^-T.  Stops when
    ||g - A^T A lambda|| <= tol ||g|| (recurrence residual; the true one is
    returned).
    """
    g = np.asarray(g, dtype=np.float64)
    D = op.D
    ng = float(np.linalg.norm(g))

    def ahat(v):
        return op.A(v / D)

    def ahat_t(u):
        return op.At(u) / D

    def prec(v):
        return solve.apply_winv(op.fac.ops, solve.apply_winvt(op.fac.ops, v))

    mu = np.zeros(op.N)
    r = g / D
    z = prec(r)
    p = z.copy()
    rho = float(r @ z)
    res = float(np.linalg.norm(D * r)) / ng if ng > 0 else 0.0
    it = 0
    while res > tol and it < max_iter:
        q = ahat_t(ahat(p))
        alpha = rho / float(p @ q)
        mu += alpha * p
        r -= alpha * q
        it += 1
        res = float(np.linalg.norm(D * r)) / ng
        z = prec(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    lam = mu / D
    true = g - op.At(op.A(lam))
    return lam, dict(iters=it, residual=float(np.linalg.norm(true)) / ng if ng > 0 else 0.0,
                     converged=res <= tol)
