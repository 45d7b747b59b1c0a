"""Pins of the oracle's analysis of matrices given without a grid
(graph nested dissection, interfaces, max-product matching; readings G1-G3
in oracle.graph_nd):

* every split is a vertex separator of G(A^T A): no edge joins the two
  children's regions, and the tree partitions the columns;
* interfaces partition their separator and nest across granularities;
* the matching is optimal: brute force over every column-to-row injection
  on tiny matrices, and it covers every column using nonzeros only;
* the factorization of a permuted grid problem is exact at eps = 0 and
  CGLS reaches the least-squares solution at eps > 0.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import graph_nd, solve, spaqr
from synth import general_ls


def _graph(p):
    return graph_nd.column_graph(p.M, p.N, np.asarray(p.row_ptr), np.asarray(p.col_idx))


@pytest.mark.parametrize("grid,depth", [((32, 32), 4), ((40, 24), 5), ((12, 12, 12), 3)])
def test_splits_are_vertex_separators(grid, depth):
    p = general_ls(grid, int(np.prod(grid)), 4)
    ptr, idx = _graph(p)
    nodes = graph_nd.build_tree(p.N, ptr, idx, depth)
    seen = np.zeros(p.N, dtype=int)
    for S in nodes:
        seen[S.sep_cols] += 1
        if S.is_leaf:
            continue
        lo, hi = S.children[0].region, S.children[1].region
        assert len(lo) and len(hi)
        side = np.zeros(p.N, dtype=int)
        side[lo] = 1
        side[hi] = 2
        for v in lo:
            assert not (side[idx[ptr[v]:ptr[v + 1]]] == 2).any()
        assert sorted(np.concatenate([lo, S.sep_cols, hi])) == sorted(S.region)
    assert (seen == 1).all()


def test_interfaces_partition_and_nest():
    p = general_ls((48, 40), 48 * 40, 5)
    ptr, idx = _graph(p)
    depth = 5
    nodes = graph_nd.build_tree(p.N, ptr, idx, depth)
    for S in nodes:
        sets = graph_nd.piece_sets(S, depth, ptr, idx, p.N)
        for g, lst in sets.items():
            cols = sorted(j for P in lst for j in P)
            assert cols == sorted(int(c) for c in S.sep_cols)
            if g + 1 in sets:
                owner = {j: k for k, P in enumerate(lst) for j in P}
                for P in sets[g + 1]:
                    assert len({owner[j] for j in P}) == 1
        if not S.is_leaf and S.level < depth - 1:
            assert len(sets[depth - 1]) > 1   # descendants cut the separator


def _brute_best(A):
    M, N = A.shape
    best = -1.0
    for rows in itertools.permutations(range(M), N):
        v = np.prod([abs(A[r, j]) for j, r in enumerate(rows)])
        best = max(best, v)
    return best


@pytest.mark.parametrize("seed", range(6))
def test_matching_is_the_max_product_one(seed):
    rng = np.random.default_rng(seed)
    M, N = 6, 4
    A = rng.standard_normal((M, N)) * (rng.random((M, N)) < 0.6)
    for j in range(N):
        if not A[:, j].any():
            A[rng.integers(M), j] = rng.standard_normal()
    S = sp.csr_matrix(A)
    S.sort_indices()
    try:
        match = graph_nd.max_product_matching(M, N, S.indptr, S.indices, S.data)
    except ValueError:
        # no matching covers every column: brute force agrees
        assert _brute_best(A) == 0.0
        return
    assert len(set(match.tolist())) == N and all(A[match[j], j] != 0 for j in range(N))
    got = np.prod([abs(A[match[j], j]) for j in range(N)])
    assert abs(got - _brute_best(A)) <= 1e-12 * got


def test_matching_on_permuted_grid_finds_the_dominant_rows():
    p = general_ls((24, 20), 480, 6)
    match = graph_nd.max_product_matching(p.M, p.N, np.asarray(p.row_ptr), np.asarray(p.col_idx),
                                          np.asarray(p.vals))
    cp, rp = p.meta["col_perm"], p.meta["row_perm"]
    # new column j is old cell cp[j]; its Laplacian row (old row cp[j]) sits at new row inv_rp[cp[j]]
    inv_rp = np.empty(p.M, dtype=np.int64)
    inv_rp[rp] = np.arange(p.M)
    lap = inv_rp[cp]
    assert np.mean(match == lap) >= 0.98


@pytest.mark.parametrize("grid,depth,skip", [((16, 16), 3, 1), ((20, 18), 4, 1)])
def test_general_exact_recovery(grid, depth, skip):
    p = general_ls(grid, int(np.prod(grid)), 7)
    an = spaqr.analyze(p, depth)
    f = spaqr.factorize(an, 0.0, skip)
    Ah = p.dense() / an.D[None, :]
    Winv = np.column_stack([solve.apply_winv(f.ops, e) for e in np.eye(an.N)])
    B = Ah @ Winv
    assert np.abs(B.T @ B - np.eye(an.N)).max() <= 1e-12
    x, info = solve.cgls(solve.Operator(f), p.b, tol=1e-13)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["iters"] <= 1 and np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_general_eps_solution():
    p = general_ls((40, 32), 1280, 8)
    an = spaqr.analyze(p, 5)
    f = spaqr.factorize(an, 1e-2, 2)
    x, info = solve.cgls(solve.Operator(f), p.b, tol=1e-12)
    xs = np.linalg.lstsq(p.dense(), p.b, rcond=None)[0]
    assert info["converged"] and np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert any(o[0] == "sparsify" for o in f.ops)
