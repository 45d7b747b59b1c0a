"""A rank-deficient grid problem for the error path of the interface
scaling (test helper; draws data only, no arithmetic of the method).

Column j2 is replaced by a copy of column j1 (same rows, same values), so
A has two identical columns and no full column rank.  Both cells sit side by
side in the top separator of a 32 x 32 grid, away from the cuts of the
lower separators, so they stay in one interface at every granularity: the
scaling QR of that interface meets two identical columns."""
import numpy as np
import scipy.sparse as sp

from synth import grid_ls


def duplicated_column_problem(seed=0):
    p = grid_ls((32, 32), 1024, seed)
    j1, j2 = 15 + 32 * 3, 16 + 32 * 3   # cells (15, 3) and (16, 3)
    A = p.scipy().tolil()
    A[:, j2] = 0
    A[:, j2] = A[:, j1]
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    A.sort_indices()
    p.row_ptr = A.indptr.astype(np.int64)
    p.col_idx = A.indices.astype(np.int32)
    p.vals = A.data.astype(np.float64)
    return p, j1, j2
