"""Pins of the inverse-Poisson generator (Appendices A and B) against the
residual it differentiates, written here independently, point by point:

2D, at interior point (i, j) with u = 0 outside the grid and z indexed on
the (n+1)^2 cell centres (z_{i,j} of the appendix is Z[i+1, j+1]):
  f = -a0 u_ij + a1 u_{i+1,j} + a2 u_{i,j+1} + a3 u_{i-1,j} + a4 u_{i,j-1}
  a0 = z_ij + z_{i-1,j} + z_{i,j-1} + z_{i-1,j-1},
  a1 = (z_ij + z_{i,j-1})/2,   a2 = (z_{i-1,j} + z_ij)/2,
  a3 = (z_{i-1,j-1} + z_{i-1,j})/2,   a4 = (z_{i,j-1} + z_{i-1,j-1})/2;
3D likewise with a0 = 3/4 of the eight surrounding cells and each face
coefficient a quarter of its four cells (sign taken positive, see the
generator).  f is linear in u for fixed z and in z for fixed u, so central
differences give its Jacobian exactly up to rounding; J^T must equal the
generator's matrix with the vanished z-rows removed.
"""
import numpy as np
import pytest

from oracle import solve, spaqr
from synth import inverse_poisson


def _f2(U, Z, n):
    def u(i, j):
        return U[i, j] if 0 <= i < n and 0 <= j < n else 0.0

    def z(i, j):  # appendix index -> cell array
        return Z[i + 1, j + 1]
    out = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            a0 = z(i, j) + z(i - 1, j) + z(i, j - 1) + z(i - 1, j - 1)
            a1 = 0.5 * (z(i, j) + z(i, j - 1))
            a2 = 0.5 * (z(i - 1, j) + z(i, j))
            a3 = 0.5 * (z(i - 1, j - 1) + z(i - 1, j))
            a4 = 0.5 * (z(i, j - 1) + z(i - 1, j - 1))
            out[i, j] = -a0 * u(i, j) + a1 * u(i + 1, j) + a2 * u(i, j + 1) + a3 * u(i - 1, j) + a4 * u(i, j - 1)
    return out


def _f3(U, Z, n):
    def u(i, j, k):
        return U[i, j, k] if 0 <= i < n and 0 <= j < n and 0 <= k < n else 0.0

    def z(i, j, k):
        return Z[i + 1, j + 1, k + 1]
    out = np.zeros((n, n, n))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                a0 = 0.75 * (z(i, j, k) + z(i - 1, j, k) + z(i, j - 1, k) + z(i, j, k - 1) + z(i - 1, j - 1, k)
                             + z(i, j - 1, k - 1) + z(i - 1, j, k - 1) + z(i - 1, j - 1, k - 1))
                a1 = 0.25 * (z(i, j, k) + z(i, j, k - 1) + z(i, j - 1, k) + z(i, j - 1, k - 1))
                a2 = 0.25 * (z(i - 1, j, k) + z(i, j, k) + z(i - 1, j, k - 1) + z(i, j, k - 1))
                a3 = 0.25 * (z(i - 1, j, k) + z(i, j, k) + z(i - 1, j - 1, k) + z(i, j - 1, k))
                a4 = 0.25 * (z(i - 1, j, k) + z(i - 1, j, k - 1) + z(i - 1, j - 1, k) + z(i - 1, j - 1, k - 1))
                a5 = 0.25 * (z(i - 1, j - 1, k) + z(i, j - 1, k) + z(i - 1, j - 1, k - 1) + z(i, j - 1, k - 1))
                a6 = 0.25 * (z(i - 1, j, k - 1) + z(i, j, k - 1) + z(i - 1, j - 1, k - 1) + z(i, j - 1, k - 1))
                out[i, j, k] = (-a0 * u(i, j, k) + a1 * u(i + 1, j, k) + a2 * u(i, j + 1, k) + a3 * u(i, j, k + 1)
                                + a4 * u(i - 1, j, k) + a5 * u(i, j - 1, k) + a6 * u(i, j, k - 1))
    return out


def _jacobian_T(p):
    n, dim = p.meta["n"], p.meta["dim"]
    U, Z = p.meta["u"], p.meta["z"]
    f = _f2 if dim == 2 else _f3

    def flat(F):  # equations numbered x fastest
        return F.ravel(order="F")
    cols = []
    h = 0.5
    for X in (U, Z):
        for idx in np.ndindex(X.shape):
            Xp, Xm = X.copy(), X.copy()
            Xp[idx] += h
            Xm[idx] -= h
            args_p = (Xp, Z) if X is U else (U, Xp)
            args_m = (Xm, Z) if X is U else (U, Xm)
            cols.append((flat(f(*args_p, n)) - flat(f(*args_m, n))) / (2 * h))
    return np.array(cols)  # rows: u then z variables, in np.ndindex order


def _reorder(JT, n, dim):
    """Rows of np.ndindex order (x slowest) -> generator order (x fastest)."""
    nu, nz = n ** dim, (n + 1) ** dim
    def perm(m):
        shape = (m,) * dim
        ids = np.arange(m ** dim).reshape(shape)          # ndindex order, last axis fastest
        return ids.transpose().ravel()                      # x fastest
    pu, pz = perm(n), perm(n + 1)
    return np.vstack([JT[:nu][pu], JT[nu:][pz]])


@pytest.mark.parametrize("dim,n,alpha", [(2, 6, 2.0), (2, 7, 1.3), (3, 4, 2.0), (3, 5, 1.6)])
def test_generator_is_the_transposed_jacobian(dim, n, alpha):
    p = inverse_poisson(n, dim, alpha, seed=3)
    JT = _reorder(_jacobian_T(p), n, dim)
    nonzero = np.abs(JT).max(axis=1) > 1e-12  # exact zeros up to the rounding of the differences
    ref = JT[nonzero]
    got = p.dense()
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(got[np.abs(ref) <= 1e-12]).max(initial=0.0) == 0.0
    # u-row c carries its largest entry, -a0, in column c
    U = got[: n ** dim]
    assert np.array_equal(np.argmax(np.abs(U), axis=1), np.arange(n ** dim))


@pytest.mark.parametrize("alpha", [2.0, 1.5, 1.05])
def test_aspect_ratio_and_solve(alpha):
    p = inverse_poisson(48, 2, alpha, seed=1)
    amin = 1 + 4 * 48 / 48 ** 2
    assert abs(p.M / p.N - max(alpha, amin)) <= 0.03
    assert (np.diff(p.row_ptr) > 0).all()
    an = spaqr.analyze(p, 5)
    f = spaqr.factorize(an, 1e-2, 2)
    x, info = solve.cgls(solve.Operator(f), p.b, tol=1e-12)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["converged"] and np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
