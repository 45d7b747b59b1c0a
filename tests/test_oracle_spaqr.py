"""Pins of the oracle factorization and solver against what the paper fixes.

* eps = 0 is the paper's "Direct" run (Section 4): the factorization is then
  exact, so (A D^-1 W^-1) has orthonormal columns, W^T W = (AD^-1)^T (AD^-1),
  CGLS converges in one iteration and x is the least-squares solution.
* The R of the first eliminated clusters is the Cholesky factor of the
  matching block of A^T A (Section 1: R equals the Cholesky factor).
* Every stored sparsification factor Q_pp is orthogonal.
* With eps > 0 the preconditioned operator stays within O(eps) of an
  isometry, and CGLS reaches the normal-equation residual bound.
* Planted mistakes in the oracle make these checks fail.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import dense, solve, spaqr
from synth import config_problem, grid_ls, CONFIGS


def _run(grid, depth, eps, skip, seed=5, extra=None):
    n = int(np.prod(grid))
    p = grid_ls(grid, n if extra is None else extra, seed)
    an = spaqr.analyze(p, depth)
    f = spaqr.factorize(an, eps, skip)
    return p, an, f


def _winv_dense(f, N):
    return np.column_stack([solve.apply_winv(f.ops, e) for e in np.eye(N)])


SMALL = [((8, 8), 2, 1), ((16, 16), 3, 1), ((16, 16), 4, 1), ((24, 20), 4, 2), ((6, 6, 6), 3, 1),
         ((8, 8, 8), 4, 1)]


@pytest.mark.parametrize("grid,depth,skip", SMALL)
def test_exact_recovery_at_eps0(grid, depth, skip):
    p, an, f = _run(grid, depth, 0.0, skip)
    Ah = p.dense() / an.D[None, :]
    Winv = _winv_dense(f, an.N)
    B = Ah @ Winv
    assert np.abs(B.T @ B - np.eye(an.N)).max() <= 1e-12
    W = np.linalg.inv(Winv)
    G = Ah.T @ Ah
    assert np.abs(W.T @ W - G).max() <= 1e-12 * np.abs(G).max()
    op = solve.Operator(f)
    x, info = solve.cgls(op, p.b, tol=1e-13)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["iters"] <= 1
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    x1 = solve.csne(op, p.b)
    assert np.linalg.norm(x1 - xs) <= 1e-12 * np.linalg.norm(xs)


def test_first_level_R_is_cholesky_factor():
    p, an, f = _run((16, 16), 4, 0.0, 1)
    Ah = p.dense() / an.D[None, :]
    G = Ah.T @ Ah
    leaves = [op for op in f.ops[:8] if op[0] == "elim"]
    assert len(leaves) == 8
    for _, s, nb, R in leaves:
        cs = s.shape[0]
        L = np.linalg.cholesky(G[np.ix_(s, s)])
        # equal up to the signs of the rows of R
        sg = np.sign(np.diag(R[:, :cs]))
        assert np.abs(sg[:, None] * R[:, :cs] - L.T).max() <= 1e-12
        assert np.abs(R[:, :cs].T @ R[:, cs:] - G[np.ix_(s, nb)]).max() <= 1e-12


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3])
def test_sparsify_factors_orthogonal_and_error_order_eps(eps):
    p, an, f = _run((32, 32), 4, eps, 1, seed=0, extra=1024)
    nsp = 0
    for op in f.ops:
        if op[0] == "sparsify":
            _, sl_, V, tau = op
            Q = np.column_stack([dense.apply_q(V, tau, e) for e in np.eye(sl_.shape[0])])
            assert np.abs(Q.T @ Q - np.eye(Q.shape[0])).max() <= 1e-13
            nsp += 1
    assert nsp > 0
    Ah = p.dense() / an.D[None, :]
    B = Ah @ _winv_dense(f, an.N)
    err = np.linalg.norm(B.T @ B - np.eye(an.N), 2)
    assert err <= 50 * eps


def test_error_decreases_with_eps():
    errs = []
    for eps in [1e-1, 1e-3, 1e-6, 0.0]:
        p, an, f = _run((24, 24), 4, eps, 1, seed=2)
        Ah = p.dense() / an.D[None, :]
        B = Ah @ _winv_dense(f, an.N)
        errs.append(np.linalg.norm(B.T @ B - np.eye(an.N), 2))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] <= 50 * 1e-3 and errs[2] <= 50 * 1e-6
    assert errs[3] <= 1e-12


def test_config1_cgls_reaches_bound_and_lstsq():
    c = CONFIGS[1]
    p = config_problem(1)
    an = spaqr.analyze(p, c["depth"])
    f = spaqr.factorize(an, c["eps"], c["skip"])
    op = solve.Operator(f)
    x, info = solve.cgls(op, p.b, tol=1e-12)
    assert info["residual"] <= 1e-12
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert 1 < info["iters"] <= 20
    # the bench tolerance
    x2, info2 = solve.cgls(op, p.b, tol=1e-10)
    A = p.dense()
    res = np.linalg.norm(A.T @ (p.b - A @ x2)) / (np.linalg.norm(A, 2) * np.linalg.norm(p.b))
    assert res <= 1e-10


def test_norm_estimate_is_lower_bound():
    p = config_problem(1)
    an = spaqr.analyze(p, 4)
    f = spaqr.factorize(an, 0.0, 1)
    est = solve.norm2_estimate(solve.Operator(f))
    exact = np.linalg.norm(p.dense(), 2)
    assert est <= exact * (1 + 1e-12) and est >= 0.99 * exact


def test_rows_never_fewer_than_columns():
    p, an, f = _run((32, 32), 4, 1e-2, 1, seed=0, extra=1024)
    for lvl, a in f.stats["aspect"]:
        assert a >= 1.0


def test_forced_ranks_reproduce_natural_run():
    p, an, f = _run((32, 32), 4, 1e-2, 1, seed=0, extra=1024)
    an2 = spaqr.analyze(p, 4)
    f2 = spaqr.factorize(an2, 1e-2, 1, forced_ranks=f.ranks)
    assert f2.ranks == f.ranks
    for a, b in zip(f.ops, f2.ops):
        assert a[0] == b[0]
        if a[0] == "elim":
            assert np.abs(a[3] - b[3]).max() <= 1e-10 * np.abs(a[3]).max()


def test_errors():
    p = grid_ls((8, 8), 10, 0)
    p.M = p.N - 1
    with pytest.raises(spaqr.SpaqrError):
        spaqr.analyze(p, 2)
    p = grid_ls((8, 8), 64, 0)
    p.vals = p.vals.copy()
    p.vals[p.col_idx == 5] = 0.0
    with pytest.raises(spaqr.SpaqrError):
        spaqr.analyze(p, 2)


# ---- planted mistakes: the pins above must catch them --------------------

def _exact_ok():
    p, an, f = _run((16, 16), 4, 0.0, 1)
    Ah = p.dense() / an.D[None, :]
    B = Ah @ _winv_dense(f, an.N)
    return np.abs(B.T @ B - np.eye(an.N)).max() <= 1e-12


def test_planted_wrong_tau_sign_is_caught(monkeypatch):
    orig = dense.house

    def bad(x):
        v, tau, beta = orig(x)
        return v, -tau, beta
    monkeypatch.setattr(dense, "house", bad)
    with pytest.raises(Exception):
        assert _exact_ok()


def test_planted_missing_right_scaling_is_caught(monkeypatch):
    monkeypatch.setattr(sl, "solve_triangular", lambda R, B, **kw: B)
    assert not _exact_ok()


def test_planted_transposed_step2_is_caught(monkeypatch):
    orig = spaqr._State.step2

    def bad(self, p, level):
        # forget to transform the neighbours' column blocks
        p1 = self.p1_of(p)
        blocks = [g for g in self.all_groups() if g is not p1 and p in g.clus]
        saved = [g.data.copy() for g in blocks]
        orig(self, p, level)
        for g, d in zip(blocks, saved):
            g.data = d
    monkeypatch.setattr(spaqr._State, "step2", bad)
    assert not _exact_ok()
