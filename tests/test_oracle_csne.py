"""Pins of the oracle's corrected seminormal equations with iterative
refinement (Section 1: the least-squares solution from W^T W x = A^T b,
with iterative refinement).

* exact factor (eps = 0): A^T A = D W^T W D exactly, so the first
  seminormal solve is already the least-squares solution (dense lstsq);
* eps > 0: every correction multiplies the error by I - M A^T A
  (M = D^-1 W^-1 W^-T D^-1); formed densely on a small grid, its spectral
  radius bounds the observed contraction of the A^T A-norm error, the
  residual history falls, and the refined x is the lstsq solution;
* a planted sign error in the correction makes the iteration diverge.
"""
import numpy as np
import pytest

from oracle import solve, spaqr
from synth import grid_ls


def _setup(grid, depth, skip, eps, seed=2):
    p = grid_ls(grid, int(np.prod(grid)), seed)
    f = spaqr.factorize(spaqr.analyze(p, depth), eps, skip)
    return p, f, solve.Operator(f)


@pytest.mark.parametrize("grid,depth", [((16, 16), 4), ((6, 6, 6), 3)])
def test_exact_factor_solves_in_one_shot(grid, depth):
    p, f, op = _setup(grid, depth, 1, 0.0)
    x, info = solve.csne_refined(op, p.b, tol=1e-12)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["steps"] == 0
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    assert np.linalg.norm(solve.csne(op, p.b) - x) <= 1e-14 * np.linalg.norm(x)


def test_refinement_contracts_by_the_iteration_matrix():
    p, f, op = _setup((16, 16), 4, 1, 1e-1)
    A = p.dense()
    AtA = A.T @ A
    N = p.N
    Mmat = np.column_stack([op.Mv(op.Mtv(e)) for e in np.eye(N)])
    G = np.eye(N) - Mmat @ AtA
    rho = max(abs(np.linalg.eigvals(G)))
    assert 0 < rho < 1
    xs = np.linalg.lstsq(A, p.b, rcond=None)[0]
    x, info = solve.csne_refined(op, p.b, tol=1e-13, max_steps=200)
    assert info["converged"]
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    h = info["history"]
    assert all(b < a for a, b in zip(h, h[1:]))
    # average contraction of the residual over the run is no better than
    # the asymptotic rate allows by much, and no worse than it
    k = info["steps"]
    assert k >= 2
    rate = (h[-1] / h[0]) ** (1.0 / k)
    assert rate <= rho * 1.5 + 1e-3
    # one correction step by hand equals (I - M A^T A) applied to the error
    x0 = op.Mv(op.Mtv(op.At(p.b)))
    x1 = x0 + op.Mv(op.Mtv(op.At(p.b - op.A(x0))))
    assert np.linalg.norm((x1 - xs) - G @ (x0 - xs)) <= 1e-10 * np.linalg.norm(x0 - xs)


def test_refinement_at_config_scale_small():
    p, f, op = _setup((32, 32), 4, 1, 1e-2, seed=0)
    x, info = solve.csne_refined(op, p.b, tol=1e-10)
    A = p.scipy()
    assert info["converged"] and info["residual"] <= 1e-10
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    assert np.linalg.norm(A.T @ (p.b - A @ x)) <= 1e-10 * info["normA"] * np.linalg.norm(p.b) * 1.0001


def test_planted_wrong_correction_sign_is_caught(monkeypatch):
    p, f, op = _setup((16, 16), 4, 1, 1e-1)
    orig = solve.Operator.Mv

    calls = {"n": 0}

    def bad(self, y):
        calls["n"] += 1
        out = orig(self, y)
        return out if calls["n"] == 1 else -out    # corrections subtracted
    monkeypatch.setattr(solve.Operator, "Mv", bad)
    x, info = solve.csne_refined(op, p.b, tol=1e-13, max_steps=20)
    assert not info["converged"]
