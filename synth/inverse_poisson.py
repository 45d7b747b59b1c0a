"""Seeded inverse-Poisson least-squares problems (the paper's Appendices A
and B): the transposed Jacobian J^T of the finite-difference residuals of
-div(z grad u) = h on an n x n (2D) or n x n x n (3D) grid of interior
points with u = 0 on the boundary, evaluated at chosen (u, z).

Columns are the equations, one per interior point (i, j[, k]), numbered
x fastest like the other grid problems, so the geometric partitioning of
the points applies.  Rows are the variables: first the u variables, in the
same order as the points (u-row c has its largest entry, -a0, in column c),
then the z variables on the (n+1)^d cell centres; z-rows that vanish are
dropped.

Stencils (cell (p, q[, r]) of z spans points p-1 .. p, q-1 .. q[, r-1 .. r],
so z_{i,j} of the appendix is cell (i+1, j+1)):

* 2D: f = -a0 u_c + a1 u_E + a2 u_N + a3 u_W + a4 u_S + q, a0 the sum of
  the four cells around the point, each a_k half the sum of the two cells
  along the face towards that neighbour;
* 3D: f = -a0 u_c + sum_k a_k u_k + q with a0 = 3/4 of the sum of the
  eight cells around the point and each a_k a quarter of the sum of the
  four cells along the face towards neighbour k.  The appendix prints the
  a_k with a minus sign; with it a constant u would not zero the
  z-derivatives that the appendix uses to shape the aspect ratio, and the
  stencil would not be the 3D analogue of the 2D one, so the sign is
  taken positive.

Values: z ~ U(1, 2) everywhere and u ~ N(0, 1), except on a centred box
of points where u = 1 (the appendix's device for lowering the aspect
ratio: every z-derivative whose stencil sees only u = 1 is exactly zero, so
its row is dropped; the appendix also sets z = 1 there, which changes no
zero pattern, and z is kept random so that the box holds no exactly
symmetric values whose ties two implementations would break differently).  The box is sized so that M / N is close to `alpha` (2 without a
box, about 1 with a box over the whole grid).  b ~ N(0, 1) of length M.
Draw order from numpy.random.default_rng(seed): z, u, b.

This module only draws problem data: it holds no arithmetic of the
factorization or of the solver.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .grid_ls import GridProblem


def _box_side(n: int, dim: int, alpha: float) -> int:
    """Side (in points) of the centred u = 1 box whose vanishing z-rows
    bring M / N closest to alpha."""
    best, best_err = 0, float("inf")
    nz = (n + 1) ** dim
    for s in range(0, n + 1):
        # a z-row's entries involve u only at its cell's 2^dim corner points,
        # so it vanishes when every corner lies in the box: (s - 1)^dim cells
        inner = max(0, s - 1) ** dim
        a = (n ** dim + nz - inner) / n ** dim
        if abs(a - alpha) < best_err:
            best, best_err = s, abs(a - alpha)
    return best


def inverse_poisson(n: int, dim: int = 2, alpha: float = 2.0, seed: int = 0) -> GridProblem:
    assert dim in (2, 3) and n >= 2
    rng = np.random.default_rng(seed)
    shape_z = (n + 1,) * dim
    z = rng.uniform(1.0, 2.0, size=shape_z)
    u = rng.standard_normal((n,) * dim)
    s = _box_side(n, dim, alpha)
    lo = (n - s) // 2
    if s > 0:
        box = tuple(slice(lo, lo + s) for _ in range(dim))
        u[box] = 1.0
    N = n ** dim
    # padded u (boundary zeros) and point numbering (x fastest)
    up = np.zeros((n + 2,) * dim)
    up[(slice(1, n + 1),) * dim] = u
    # arrays are indexed [x, y(, z)]
    if dim == 2:
        I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        col = (I + n * J).ravel()
        pts = [I.ravel(), J.ravel()]
    else:
        I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        col = (I + n * (J + n * K)).ravel()
        pts = [I.ravel(), J.ravel(), K.ravel()]
    rows, cols, vals = [], [], []

    def point_id(ix):
        if dim == 2:
            return ix[0] + n * ix[1]
        return ix[0] + n * (ix[1] + n * ix[2])

    def zcell(c):  # cell index -> z row index (after the n^dim u rows)
        if dim == 2:
            return N + c[0] + (n + 1) * c[1]
        return N + c[0] + (n + 1) * (c[1] + (n + 1) * c[2])

    def uval(ix):  # u at point offsets (0 outside the grid)
        return up[tuple(a + 1 for a in ix)]

    # cells around point p: offsets d in {0,1}^dim, cell = p + d (cell p+1
    # is the appendix's z_{p}); faces towards neighbour e (+-1 along axis)
    corners = [tuple((m >> a) & 1 for a in range(dim)) for m in range(2 ** dim)]
    ccoef = 1.0 if dim == 2 else 0.75   # weight of each cell in a0
    fcoef = 0.5 if dim == 2 else 0.25   # weight of each cell in a face coefficient
    zc = {d: z[tuple(pts[a] + d[a] for a in range(dim))] for d in corners}
    a0 = ccoef * sum(zc[d] for d in corners)
    # u derivatives: -a0 on the point, a_e on in-grid neighbours
    rows.append(col)
    cols.append(col)
    vals.append(-a0)
    for axis in range(dim):
        for sgn in (1, -1):
            # cells on the face towards the neighbour: offset along axis is 1
            # for +1, 0 for -1; free along the other axes
            face = [d for d in corners if d[axis] == (1 if sgn > 0 else 0)]
            ae = fcoef * sum(zc[d] for d in face)
            nb = [p.copy() for p in pts]
            nb[axis] = nb[axis] + sgn
            ok = (nb[axis] >= 0) & (nb[axis] < n)
            rows.append(point_id([q[ok] for q in nb]))
            cols.append(col[ok])
            vals.append(ae[ok])
    # z derivatives: cell p + d appears in a0 (weight ccoef, times -u_p) and
    # in the faces towards the neighbours p + e for which d lies on that face
    for d in corners:
        g = -ccoef * uval(pts)
        for axis in range(dim):
            sgn = 1 if d[axis] == 1 else -1
            nb = [p.copy() for p in pts]
            nb[axis] = nb[axis] + sgn
            g = g + fcoef * uval(nb)
        cell = [pts[a] + d[a] for a in range(dim)]
        rows.append(zcell(cell))
        cols.append(col)
        vals.append(g)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    Mfull = N + (n + 1) ** dim
    A = sp.csr_matrix((v, (r, c)), shape=(Mfull, N))
    A.sum_duplicates()
    A.eliminate_zeros()
    keep = np.diff(A.indptr) > 0
    A = A[np.flatnonzero(keep)]
    A.sort_indices()
    M = A.shape[0]
    b = rng.standard_normal(M)
    p = GridProblem(grid=(n, n, 1) if dim == 2 else (n, n, n), M=M, N=N,
                    row_ptr=A.indptr.astype(np.int64), col_idx=A.indices.astype(np.int32),
                    vals=A.data.astype(np.float64), b=b, seed=seed)
    p.meta = dict(kind="inverse_poisson", n=n, dim=dim, alpha_target=alpha, alpha=M / N, box=s,
                  u=u, z=z)
    return p
