"""Pins of the oracle on square systems (M = N), the spaQR of Section 2.1:
with one matched row per column every cluster keeps as many rows as
columns, so no rows fall below a diagonal (nothing to reassign, nothing
for sparsification step 1) and only step 2 sparsifies.

* exact recovery at eps = 0: (A D^-1 W^-1) is orthogonal, W^T W = Ahat^T Ahat,
  x = A^-1 b in one CGLS iteration;
* eps > 0: only step-2 rank-revealing QRs occur, every Q_pp is orthogonal,
  the error of W^T W is O(eps) and shrinks with eps, and CGLS reaches
  the solution of the linear system;
* the first-level R factors are the Cholesky factors of Ahat^T Ahat's
  diagonal blocks (up to row signs)."""
import numpy as np
import pytest

from oracle import dense, solve, spaqr
from synth import grid_square


def _run(grid, depth, eps, skip, seed=3):
    p = grid_square(grid, seed)
    an = spaqr.analyze(p, depth)
    log = []
    f = spaqr.factorize(an, eps, skip, log=log)
    return p, an, f, log


def _winv_dense(f, N):
    return np.column_stack([solve.apply_winv(f.ops, e) for e in np.eye(N)])


@pytest.mark.parametrize("grid,depth,skip", [((16, 16), 4, 1), ((6, 6, 6), 3, 1), ((17, 13), 4, 1)])
def test_square_exact_recovery(grid, depth, skip):
    p, an, f, log = _run(grid, depth, 0.0, skip)
    assert p.M == p.N
    Ah = p.dense() / an.D[None, :]
    B = Ah @ _winv_dense(f, an.N)
    assert np.abs(B.T @ B - np.eye(an.N)).max() <= 1e-11
    x, info = solve.cgls(solve.Operator(f), p.b, tol=1e-13)
    xs = np.linalg.solve(p.dense(), p.b)
    assert info["iters"] <= 1
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_square_only_step2_and_first_level_cholesky():
    p, an, f, log = _run((32, 32), 4, 1e-2, 1)
    assert log and all(r["kind"] == "step2" for r in log)
    Ah = p.dense() / an.D[None, :]
    G = Ah.T @ Ah
    leaves = [op for op in f.ops if op[0] == "elim"][:8]
    for _, s, nb, R in leaves:
        cs = s.shape[0]
        L = np.linalg.cholesky(G[np.ix_(s, s)])
        sg = np.sign(np.diag(R[:, :cs]))
        assert np.abs(sg[:, None] * R[:, :cs] - L.T).max() <= 1e-11 * np.abs(L).max()
    for op in f.ops:
        if op[0] == "sparsify":
            _, pp, V, tau = op
            Q = dense.apply_q(V, tau, np.eye(V.shape[0]))
            assert np.abs(Q.T @ Q - np.eye(V.shape[0])).max() <= 1e-13


def test_square_error_order_eps_and_solution():
    errs = []
    for eps in (1e-1, 1e-2, 1e-3):
        p, an, f, log = _run((24, 24), 4, eps, 1)
        Ah = p.dense() / an.D[None, :]
        B = Ah @ _winv_dense(f, an.N)
        e = np.linalg.norm(B.T @ B - np.eye(an.N), 2)
        errs.append(e)
        x, info = solve.cgls(solve.Operator(f), p.b, tol=1e-12)
        xs = np.linalg.solve(p.dense(), p.b)
        assert info["converged"] and np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] <= 100 * 1e-2
