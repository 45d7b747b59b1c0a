"""Pins of the oracle's dense kernels against LAPACK (numpy / scipy).

numpy.linalg.qr runs LAPACK dgeqrf, whose reflectors follow the same sign
convention (beta = -sign(alpha) ||x||), so R must agree entry by entry, signs
included.  scipy.linalg.qr(pivoting=True) runs dgeqp3, the same greedy
max-column-norm pivoting family as the dlaqps routine the paper names
(Section 4), so pivots and R must agree on matrices without near ties.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import dense


@pytest.mark.parametrize("m,n", [(50, 30), (30, 30), (7, 12), (1, 5), (64, 1)])
def test_householder_matches_lapack(m, n):
    rng = np.random.default_rng(m * 100 + n)
    A = rng.standard_normal((m, n))
    F = A.copy()
    refl = dense.householder_qr(F)
    k = min(m, n)
    R = np.linalg.qr(A, mode="r")
    assert np.abs(np.triu(F[:k]) - R[:k]).max() <= 1e-13 * np.abs(A).max()
    # Q built from the reflectors is orthogonal and reproduces A
    Q = np.eye(m)
    for i in range(len(refl) - 1, -1, -1):
        v, tau = refl[i]
        Q[i:, :] -= tau * np.outer(v, v @ Q[i:, :])
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 1e-14 * m
    assert np.abs(Q @ np.triu(F) - A).max() <= 1e-13 * np.abs(A).max() * max(m, n)


def test_householder_trailing_columns_only_first_block():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 25))
    F = A.copy()
    dense.householder_qr(F, 10)
    # first 10 columns factored; Q^T applied to the other 15
    Qf, Rf = np.linalg.qr(A[:, :10], mode="complete")
    assert np.allclose(np.triu(F[:10, :10]), Rf[:10], atol=1e-13)
    assert np.allclose(F[:, 10:], Qf.T @ A[:, 10:], atol=1e-12)


def test_house_zero_tail_is_identity():
    v, tau, beta = dense.house(np.array([3.0, 0.0, 0.0]))
    assert tau == 0.0 and beta == 3.0
    v, tau, beta = dense.house(np.array([0.0, 3.0, 4.0]))
    assert beta == -5.0  # sign(0) = +1


def _separated(m, n, seed, spread=4.0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, n)) * np.logspace(0, -spread, n)[None, :]
    return B[:, rng.permutation(n)]


@pytest.mark.parametrize("m,n,seed", [(40, 25, 0), (25, 40, 1), (60, 60, 2), (5, 30, 3)])
def test_pivoted_matches_lapack_geqp3(m, n, seed):
    B = _separated(m, n, seed)
    r, rows, perm, V, tau = dense.pivoted_qr(B, 0.0)
    Q, R, P = sl.qr(B, pivoting=True)
    k = min(m, n)
    assert r == k
    assert (perm == P[:k]).all()
    assert np.abs(rows[:, P] - np.triu(R)[:k]).max() <= 1e-13 * np.abs(B).max()
    # rows are Q^T B in the original column order; Q from the reflectors matches
    assert np.abs(dense.apply_qt(V, tau, B)[:r] - rows).max() <= 1e-13 * np.abs(B).max()


def test_pivoted_downdate_recompute_path():
    # strongly correlated columns: norm downdates cancel and must be recomputed
    rng = np.random.default_rng(7)
    base = rng.standard_normal((30, 1))
    B = base + 1e-9 * rng.standard_normal((30, 12)) * np.logspace(0, -2, 12)[None, :]
    r, rows, perm, V, tau = dense.pivoted_qr(B, 0.0)
    Q, R, P = sl.qr(B, pivoting=True)
    assert (perm[:6] == P[:6]).all()


def test_rank_rule_closed_form():
    # orthogonal columns with known norms: |R_ii| are the sorted norms, so the
    # rank rule keeps exactly the norms >= eps * max norm
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 8)))
    norms = np.array([1.0, 3e-3, 0.5, 2e-1, 1e-5, 7e-2, 9e-3, 4e-4])
    C = Q * norms[None, :]
    for eps, expect in [(1e-1, 3), (1e-2, 4), (5e-3, 5), (1e-3, 6), (1e-4, 7), (1e-6, 8), (0.0, 8)]:
        r, rows, perm, V, tau = dense.pivoted_qr(C, eps)
        assert r == expect, (eps, r)
        assert list(perm) == list(np.argsort(-norms)[:expect])
        # the dropped part of Q^T C has the size of the dropped norms
        full = dense.apply_qt(V, tau, C)
        assert np.linalg.norm(full[r:]) <= 1.0001 * np.linalg.norm(np.sort(norms)[::-1][r:]) + 1e-15


def test_rank_zero_for_zero_and_empty():
    assert dense.pivoted_qr(np.zeros((5, 4)), 1e-2)[0] == 0
    assert dense.pivoted_qr(np.zeros((5, 0)), 1e-2)[0] == 0
    assert dense.pivoted_qr(np.zeros((0, 4)), 1e-2)[0] == 0


def test_rounding_level_alpha_takes_the_positive_sign():
    """An alpha that is a structural zero carrying rounding error (either
    sign) gives the same reflector as an exact zero; a genuinely small alpha
    above the floor keeps its sign."""
    tail = np.array([0.3, -1.2, 0.5])
    ref = dense.house(np.concatenate([[0.0], tail]))
    for a in (1e-22, -1e-22, -4e-17):
        v, tau, beta = dense.house(np.concatenate([[a], tail]))
        assert beta < 0 and abs(beta - ref[2]) <= 1e-15 and abs(tau - ref[1]) <= 1e-15
    v, tau, beta = dense.house(np.concatenate([[-1e-9], tail]))
    assert beta > 0
    # the same front column with structural-zero noise of opposite signs
    F = np.array([[-3e-21, 1.0], [0.6, 2.0], [0.8, -1.0]])
    G = F.copy()
    G[0, 0] = 3e-21
    dense.householder_qr(F)
    dense.householder_qr(G)
    assert np.abs(np.triu(F[:2]) - np.triu(G[:2])).max() <= 1e-15

