"""Pins of the oracle's partitioning (Section 2.2, Figure 3)."""
import os

import numpy as np
import pytest

from oracle import nd, spaqr
from synth import grid_ls

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "nd_grid32x32_depth4.txt")


def _cells(lo, hi, grid):
    return set(nd.box_cells(lo, hi, grid))


@pytest.mark.parametrize("grid,depth", [((32, 32, 1), 4), ((17, 23, 1), 3), ((256, 256, 1), 8),
                                        ((12, 10, 9), 4), ((32, 32, 32), 6)])
def test_tree_partitions_every_cell_once(grid, depth):
    nodes = nd.build_tree(grid, depth)
    seen = set()
    total = 0
    for S in nodes:
        lo, hi = S.sep_box(2)
        cells = _cells(lo, hi, grid)
        total += len(cells)
        assert not (seen & cells)
        seen |= cells
        if not S.is_leaf:
            assert hi[S.axis] - lo[S.axis] == 2
            # the two children lie on either side of the separator, same face extent
            a = S.axis
            c0, c1 = S.children
            assert c0.hi[a] == S.t and c1.lo[a] == S.t + 2
    assert total == grid[0] * grid[1] * grid[2] and len(seen) == total
    assert sum(1 for S in nodes if S.is_leaf) == 2 ** (depth - 1)
    ranks = [S.rank for S in nodes]
    assert ranks == list(range(len(nodes)))


def test_golden_grid32x32_depth4():
    grid = (32, 32, 1)
    nodes = nd.build_tree(grid, 4)
    by = {(S.level, S.path): S for S in nodes}
    root_pieces = []
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "root_g2":
            v = list(map(int, tok[1:]))
            root_pieces.append((tuple(v[:3]), tuple(v[3:])))
            continue
        left, right = line.split("|")
        lv, path, axis, t, *box = map(int, left.split())
        S = by[(lv, path)]
        assert (S.axis, S.t) == (axis, t)
        assert S.lo == tuple(box[:3]) and S.hi == tuple(box[3:])
        for item in right.split():
            g, cnt = item[1:].split(":")
            assert len(nd.pieces(S, int(g))) == int(cnt), (lv, path, g)
    root = by[(1, 0)]
    assert sorted(nd.pieces(root, 2)) == sorted(root_pieces)


@pytest.mark.parametrize("grid,depth", [((32, 32, 1), 4), ((64, 48, 1), 6), ((16, 16, 16), 5)])
def test_pieces_nest_and_cover(grid, depth):
    nodes = nd.build_tree(grid, depth)
    for S in nodes:
        if S.is_leaf:
            continue
        lo, hi = S.sep_box(2)
        whole = _cells(lo, hi, grid)
        prev = None
        for g in range(S.level, nd.finest_granularity(S, depth) + 1):
            ps = nd.pieces(S, g)
            sets = [_cells(a, b, grid) for a, b in ps]
            assert set().union(*sets) == whole and sum(map(len, sets)) == len(whole)
            if prev is not None:
                for s in sets:
                    assert sum(1 for q in prev if s <= q) == 1
            prev = sets


def test_two_plane_separators_separate_rows():
    # every row of the generated problems stays inside one root-to-leaf path
    for grid, d in [((32, 32), 4), ((20, 20, 20), 4)]:
        p = grid_ls(grid, p_extra := grid[0] * grid[1] * (grid[2] if len(grid) > 2 else 1) // 2, 9)
        spaqr.analyze(p, d)  # raises if a row touches two sibling subtrees


def test_one_plane_separator_is_rejected():
    # radius-1 rows couple cells at distance 2: a single plane cannot separate
    p = grid_ls((32, 32), 1024, 0)
    with pytest.raises(spaqr.SpaqrError):
        spaqr.analyze(p, 4, w=1)


def test_row_ownership_max_norm_rule():
    p = grid_ls((24, 24), 576, 5)
    an = spaqr.analyze(p, 4)
    A = p.dense() / an.D[None, :]
    owner = an.row_owner
    # matched rows: the Laplacian row of a cell belongs to the cell's cluster
    for j in range(an.N):
        assert an.finest[owner[j]] is an.col_cluster[j]
    # other rows: no cluster holds more of the row's squared norm than the owner
    cl = np.array([an.col_cluster[j].index for j in range(an.N)])
    for r in range(an.N, an.M):
        mass = np.bincount(cl, weights=A[r] ** 2, minlength=len(an.finest))
        assert mass[owner[r]] == mass.max()
        assert owner[r] == int(np.flatnonzero(mass == mass.max())[0])
