"""Seeded synthetic grid least-squares problems.

This module only draws problem data.  It holds no arithmetic of the
factorization or of the solver, so both the FP64 CPU oracle and the GPU path
can take their inputs from it without sharing any of the method.

Problem recipe (stands in for the PDE-constrained Jacobians of the paper's
Section 4: same grid structure, local row supports, aspect ratio about 2 in
2D and 1.5 in 3D):

* cells ``k = i + nx*(j + ny*l)`` (x fastest), one column per cell;
* rows ``0..N-1``: Laplacian rows with Dirichlet boundary (2D: 4 on the
  diagonal and -1 on in-grid 4-neighbours; 3D: 6 and -1 on 6-neighbours);
* rows ``N..M-1``: random local rows.  Per row an anchor cell is drawn; in 2D
  the row holds the anchor plus the two in-grid 4-neighbours with the
  smallest random keys (neighbour slots ordered -x,+x,-y,+y); in 3D it holds
  the four in-grid cells of the clipped 3x3x3 box around the anchor (anchor
  included, slots ordered with x fastest) with the smallest keys.  Values are
  standard normal, assigned to the sorted columns in order;
* ``b`` standard normal of length M, then (when asked) a target ``x_t`` of
  length N.

Draw order from ``numpy.random.default_rng(seed)``: anchors, keys, values,
b, x_t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class GridProblem:
    grid: tuple            # (nx, ny, nz); nz == 1 for 2D
    M: int
    N: int
    row_ptr: np.ndarray    # int64, M+1
    col_idx: np.ndarray    # int32, nnz (sorted within each row)
    vals: np.ndarray       # float64, nnz
    b: np.ndarray          # float64, M
    x_t: np.ndarray | None = None
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        A = np.zeros((self.M, self.N))
        for r in range(self.M):
            lo, hi = self.row_ptr[r], self.row_ptr[r + 1]
            A[r, self.col_idx[lo:hi]] = self.vals[lo:hi]
        return A

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.M, self.N))


def _laplacian(nx, ny, nz):
    N = nx * ny * nz
    k = np.arange(N)
    i = k % nx
    j = (k // nx) % ny
    l = k // (nx * ny)
    dim3 = nz > 1
    diag = 6.0 if dim3 else 4.0
    rows = [k]
    cols = [k]
    vals = [np.full(N, diag)]
    nbrs = [(i > 0, -1), (i < nx - 1, 1), (j > 0, -nx), (j < ny - 1, nx)]
    if dim3:
        nbrs += [(l > 0, -nx * ny), (l < nz - 1, nx * ny)]
    for mask, off in nbrs:
        rows.append(k[mask])
        cols.append(k[mask] + off)
        vals.append(np.full(int(mask.sum()), -1.0))
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def grid_ls(grid, extra_rows: int, seed: int, with_target: bool = False) -> GridProblem:
    """Draw one problem on ``grid`` = (nx, ny) or (nx, ny, nz)."""
    if len(grid) == 2:
        grid = (int(grid[0]), int(grid[1]), 1)
    nx, ny, nz = (int(g) for g in grid)
    N = nx * ny * nz
    R = int(extra_rows)
    M = N + R
    dim3 = nz > 1
    rng = np.random.default_rng(seed)

    lr, lc, lv = _laplacian(nx, ny, nz)

    anchors = rng.integers(0, N, size=R)
    ai = anchors % nx
    aj = (anchors // nx) % ny
    al = anchors // (nx * ny)
    if not dim3:
        offs = np.array([[-1, 0], [1, 0], [0, -1], [0, 1]])  # (dx, dy): -x,+x,-y,+y
        keys = rng.random((R, 4))
        ci = ai[:, None] + offs[None, :, 0]
        cj = aj[:, None] + offs[None, :, 1]
        ok = (ci >= 0) & (ci < nx) & (cj >= 0) & (cj < ny)
        keys = np.where(ok, keys, np.inf)
        pick = np.argsort(keys, axis=1, kind="stable")[:, :2]
        pi = np.take_along_axis(ci, pick, 1)
        pj = np.take_along_axis(cj, pick, 1)
        ecols = np.concatenate([anchors[:, None], pi + nx * pj], axis=1)
        nper = 3
    else:
        d = np.arange(-1, 2)
        dz, dy, dx = np.meshgrid(d, d, d, indexing="ij")  # x fastest in the flattened order
        offs = np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=1)  # 27 slots
        keys = rng.random((R, 27))
        ci = ai[:, None] + offs[None, :, 0]
        cj = aj[:, None] + offs[None, :, 1]
        cl = al[:, None] + offs[None, :, 2]
        ok = (ci >= 0) & (ci < nx) & (cj >= 0) & (cj < ny) & (cl >= 0) & (cl < nz)
        keys = np.where(ok, keys, np.inf)
        pick = np.argsort(keys, axis=1, kind="stable")[:, :4]
        ecols = (np.take_along_axis(ci, pick, 1) + nx * (np.take_along_axis(cj, pick, 1)
                 + ny * np.take_along_axis(cl, pick, 1)))
        nper = 4
    ecols = np.sort(ecols, axis=1)
    evals = rng.standard_normal((R, nper))
    b = rng.standard_normal(M)
    x_t = rng.standard_normal(N) if with_target else None

    # assemble CSR: Laplacian rows (sorted columns) then the random rows
    order = np.lexsort((lc, lr))
    lr, lc, lv = lr[order], lc[order], lv[order]
    lap_counts = np.bincount(lr, minlength=N)
    row_ptr = np.zeros(M + 1, dtype=np.int64)
    row_ptr[1:N + 1] = np.cumsum(lap_counts)
    row_ptr[N + 1:] = row_ptr[N] + nper * np.arange(1, R + 1)
    col_idx = np.concatenate([lc, ecols.ravel()]).astype(np.int32)
    vals = np.concatenate([lv, evals.ravel()]).astype(np.float64)
    return GridProblem(grid=(nx, ny, nz), M=M, N=N, row_ptr=row_ptr, col_idx=col_idx,
                       vals=vals, b=b, x_t=x_t, seed=seed)


def general_ls(grid, extra_rows: int, seed: int, jitter: float = 0.1) -> GridProblem:
    """A grid problem handed over as a general sparse matrix: rows and
    columns in random order, no grid attached (grid None), and the
    Laplacian rows' values jittered by jitter * N(0, 1) so that no two
    entries tie.  Draw order: the grid problem's draws (seed), then from
    default_rng(seed + 7919): the column permutation, the row permutation,
    the jitter.  meta keeps both permutations (col_perm[new] = old column,
    row_perm[new] = old row)."""
    p = grid_ls(grid, extra_rows, seed)
    rng = np.random.default_rng(seed + 7919)
    cp = rng.permutation(p.N)
    rp = rng.permutation(p.M)
    vals = p.vals.copy()
    nlap = int(p.row_ptr[p.N])
    vals[:nlap] += jitter * rng.standard_normal(nlap)
    inv = np.empty(p.N, dtype=np.int64)
    inv[cp] = np.arange(p.N)
    A = p.scipy().tocoo()
    rows_new = np.empty(p.M, dtype=np.int64)
    rows_new[rp] = np.arange(p.M)
    import scipy.sparse as sp
    B = sp.csr_matrix((vals, (rows_new[A.row], inv[A.col])), shape=(p.M, p.N))
    B.sort_indices()
    q = GridProblem(grid=None, M=p.M, N=p.N, row_ptr=B.indptr.astype(np.int64),
                    col_idx=B.indices.astype(np.int32), vals=B.data.astype(np.float64), b=p.b[rp].copy(),
                    seed=seed)
    q.meta = dict(kind="general", col_perm=cp, row_perm=rp, source_grid=tuple(p.grid))
    return q


def grid_square(grid, seed: int, skew: float = 0.3) -> GridProblem:
    """Square nonsymmetric grid system (M = N): the Laplacian's stencil
    pattern with off-diagonal values -1 + skew * N(0,1), drawn independently
    for (i, j) and (j, i), and each diagonal equal to the sum of the
    magnitudes of its row's off-diagonals plus one per out-of-grid neighbour
    (weakly diagonally dominant, strictly on rows next to the Dirichlet
    boundary, irreducible: nonsingular);
    b standard normal.  Draw order: off-diagonal values, b."""
    if len(grid) == 2:
        grid = (int(grid[0]), int(grid[1]), 1)
    nx, ny, nz = (int(g) for g in grid)
    N = nx * ny * nz
    rng = np.random.default_rng(seed)
    lr, lc, lv = _laplacian(nx, ny, nz)
    order = np.lexsort((lc, lr))
    lr, lc = lr[order], lc[order]
    off = lr != lc
    vals = np.zeros(lr.shape[0])
    vals[off] = -1.0 + skew * rng.standard_normal(int(off.sum()))
    rowsum = np.bincount(lr, weights=np.abs(vals), minlength=N)
    nbrs = np.bincount(lr[off], minlength=N)
    # missing (out-of-grid) neighbours count 1 each, as in the Dirichlet Laplacian
    vals[~off] = rowsum[lr[~off]] + (6 if nz > 1 else 4) - nbrs[lr[~off]]
    b = rng.standard_normal(N)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(np.bincount(lr, minlength=N))
    return GridProblem(grid=(nx, ny, nz), M=N, N=N, row_ptr=row_ptr, col_idx=lc.astype(np.int32),
                       vals=vals, b=b, seed=seed)


def default_depth(N: int) -> int:
    """Tree levels ceil(log2(N/64)) (Section 4), at least 2."""
    return max(2, int(math.ceil(math.log2(N / 64.0))))


# The five benchmark configurations.  ``depth`` counts tree levels including
# the leaf level; ``skip`` is the number of leaf-side levels that are not
# sparsified (Section 4: sparsification starts on level 3 or 4).
CONFIGS = {
    1: dict(name="grid2d_32x32", grid=(32, 32), extra=1024, seed=0, depth=4, eps=1e-2, skip=1),
    2: dict(name="grid2d_256x256", grid=(256, 256), extra=65536, seed=1, depth=8, eps=1e-3, skip=2),
    3: dict(name="grid3d_32x32x32", grid=(32, 32, 32), extra=16384, seed=2, depth=6, eps=1e-2, skip=2),
    5: dict(name="grid2d_128x128_grad", grid=(128, 128), extra=16384, seed=4, depth=8, eps=1e-2, skip=2,
            target=True),
}


def config_problem(cfg: int) -> GridProblem:
    c = CONFIGS[cfg]
    p = grid_ls(c["grid"], c["extra"], c["seed"], with_target=c.get("target", False))
    p.meta = dict(c)
    return p


def batch_sides(count: int = 64) -> np.ndarray:
    """Side lengths of the batch of independent 2D problems (48..160)."""
    return np.random.default_rng(3).integers(48, 161, count)


def batch_problem(i: int, sides=None) -> GridProblem:
    """Problem i of the batch: s x s grid, M = 2N, seed 100+i."""
    if sides is None:
        sides = batch_sides()
    s = int(sides[i])
    p = grid_ls((s, s), s * s, 100 + i)
    p.meta = dict(name=f"batch{i}_{s}x{s}", grid=(s, s), depth=default_depth(s * s), eps=1e-2, skip=2)
    return p
