"""Pins of the adjoint oracle (CPU only).

* central finite differences of L = 0.5 ||x*(A, b) - x_t||^2, with x* from
  dense LAPACK least squares (no normal equations), against the gradient
  formula for b and for sampled nonzeros of A;
* dL/db against the pseudo-inverse closed form pinv(A)^T g;
* a planted dropped term (the r_i lambda_j part) must fail the FD check;
* lambda from the spaQR-preconditioned CG against the direct solve.
"""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import solve as osolve
from oracle import spaqr as osp
from synth import grid_ls


def _small(seed=5, grid=(10, 8)):
    n = grid[0] * grid[1]
    return grid_ls(grid, n, seed, with_target=True)


def _loss(p, vals, b):
    A = np.zeros((p.M, p.N))
    rows = np.repeat(np.arange(p.M), np.diff(p.row_ptr))
    A[rows, p.col_idx] = vals
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    return 0.5 * float(np.sum((x - p.x_t) ** 2)), x


def _fd_check(p, gb, gv, picks_v, picks_b, h=1e-6):
    worst = 0.0
    scale = max(np.abs(gv).max(), np.abs(gb).max())
    for e in picks_v:
        vp, vm = p.vals.copy(), p.vals.copy()
        vp[e] += h
        vm[e] -= h
        fd = (_loss(p, vp, p.b)[0] - _loss(p, vm, p.b)[0]) / (2 * h)
        worst = max(worst, abs(fd - gv[e]) / scale)
    for i in picks_b:
        bp, bm = p.b.copy(), p.b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (_loss(p, p.vals, bp)[0] - _loss(p, p.vals, bm)[0]) / (2 * h)
        worst = max(worst, abs(fd - gb[i]) / scale)
    return worst


def _grads(p):
    x = oadj.lstsq_solution(p.row_ptr, p.col_idx, p.vals, p.b, p.M, p.N)
    g = x - p.x_t
    gb, gv, lam = oadj.grads_direct(p.row_ptr, p.col_idx, p.vals, p.b, x, g, p.M, p.N)
    return x, g, gb, gv, lam


def test_solution_matches_dense_lstsq():
    p = _small()
    x = oadj.lstsq_solution(p.row_ptr, p.col_idx, p.vals, p.b, p.M, p.N)
    xd = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert np.abs(x - xd).max() <= 1e-12 * np.abs(xd).max()


def test_gradients_match_finite_differences():
    p = _small()
    _, _, gb, gv, _ = _grads(p)
    rng = np.random.default_rng(11)
    picks_v = rng.choice(p.nnz, 20, replace=False)
    picks_b = rng.choice(p.M, 10, replace=False)
    assert _fd_check(p, gb, gv, picks_v, picks_b) <= 1e-6


def test_grad_b_is_pinv_transpose_g():
    p = _small(seed=6, grid=(7, 9))
    x, g, gb, _, _ = _grads(p)
    ref = np.linalg.pinv(p.dense()).T @ g
    assert np.abs(gb - ref).max() <= 1e-11 * np.abs(ref).max()


def test_planted_dropped_term_is_caught():
    p = _small(seed=7)
    x, g, gb, gv, lam = _grads(p)
    rows = np.repeat(np.arange(p.M), np.diff(p.row_ptr))
    Al = p.scipy() @ lam
    wrong = -Al[rows] * x[p.col_idx]        # the r_i lambda_j term dropped
    rng = np.random.default_rng(12)
    picks = rng.choice(p.nnz, 20, replace=False)
    assert _fd_check(p, gb, wrong, picks, []) > 1e-3


@pytest.mark.parametrize("eps", [1e-2, 1e-1])
def test_pcg_adjoint_matches_direct(eps):
    p = grid_ls((16, 16), 256, 8, with_target=True)
    an = osp.analyze(p, 4)
    f = osp.factorize(an, eps, 1)
    op = osolve.Operator(f)
    x, g, _, _, lam = _grads(p)
    lp, info = oadj.adjoint_pcg(op, g, tol=1e-13)
    assert info["converged"] and info["residual"] <= 1e-12
    assert np.abs(lp - lam).max() <= 1e-10 * np.abs(lam).max()
    # a good preconditioner: few iterations, fewer for the finer eps
    assert info["iters"] <= 30
