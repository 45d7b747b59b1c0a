"""Geometric nested dissection, interfaces and cluster hierarchy (oracle).

Test infrastructure only.  Restates Section 2.2 (partitioning; the paper
allows a geometric partition when the grid is known, Section 4.1) with these
readings:

* tree levels 1 (root) .. d (leaves); a box at level < d is split across its
  longest axis (ties: x before y before z) by a separator of ``w`` (default
  2) consecutive cell planes starting at ``lo + (len - w) // 2``; low child
  first.  Two planes are needed because a row reaches cells at distance 1,
  so G(A^T A) couples cells up to distance 2;
* interfaces of a separator S (level l) at granularity g (l <= g <= d-1):
  along each face axis of S, start from S's extent and, for every level
  lambda = l+1..g, split every current interval into maximal runs of cells
  that are / are not covered by the cut planes of the level-lambda
  descendant separators whose boxes touch S and which split along that
  axis.  Pieces are the tensor products of the per-axis intervals, so the
  pieces at g+1 nest in those at g (the cluster hierarchy of Figure 3);
* cluster order ("id"): separators in elimination order (leaves first, in
  left-to-right tree order, then each level up to the root), and pieces of
  one separator by the cell index of their lower corner.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(eq=False)
class NDNode:
    level: int
    path: int
    lo: tuple
    hi: tuple
    axis: int = -1           # split axis, -1 for a leaf
    t: int = -1              # first separator plane along ``axis``
    children: list = field(default_factory=list)
    parent: "NDNode | None" = None
    rank: int = -1           # elimination rank (leaves first)

    @property
    def is_leaf(self) -> bool:
        return self.axis < 0

    def sep_box(self, w):
        lo = list(self.lo)
        hi = list(self.hi)
        if not self.is_leaf:
            lo[self.axis] = self.t
            hi[self.axis] = self.t + w
        return tuple(lo), tuple(hi)

    def subtree(self):
        out = [self]
        for c in self.children:
            out.extend(c.subtree())
        return out


def build_tree(grid, depth: int, w: int = 2) -> list:
    """Build the ND tree; returns all nodes sorted by elimination rank."""
    grid = tuple(grid) + (1,) * (3 - len(grid))

    def rec(lo, hi, level, path, parent):
        node = NDNode(level=level, path=path, lo=lo, hi=hi, parent=parent)
        if level < depth:
            lens = [hi[a] - lo[a] for a in range(3)]
            axis = max(range(3), key=lambda a: (lens[a], -a))
            L = lens[axis]
            if L < w + 2:
                raise ValueError(f"box {lo}-{hi} too small to split at level {level}")
            t = lo[axis] + (L - w) // 2
            node.axis, node.t = axis, t
            lhi = list(hi)
            lhi[axis] = t
            hlo = list(lo)
            hlo[axis] = t + w
            node.children = [rec(lo, tuple(lhi), level + 1, 2 * path, node),
                             rec(tuple(hlo), hi, level + 1, 2 * path + 1, node)]
        return node

    root = rec((0, 0, 0), grid, 1, 0, None)
    nodes = root.subtree()
    nodes.sort(key=lambda n: (-n.level, n.path))
    for i, n in enumerate(nodes):
        n.rank = i
    return nodes


def _touching_cuts(S: NDNode, level: int, axis_b: int, w: int):
    """Cut cell set along ``axis_b`` from level-``level`` descendants of S."""
    a = S.axis
    cuts = set()
    for T in S.subtree():
        if T is S or T.level != level or T.is_leaf or T.axis != axis_b:
            continue
        if T.hi[a] == S.t or T.lo[a] == S.t + w:
            cuts.update(range(T.t, T.t + w))
    return cuts


def _refine(intervals, cuts):
    out = []
    for (a0, a1) in intervals:
        start = a0
        for c in range(a0 + 1, a1):
            if (c in cuts) != (c - 1 in cuts):
                out.append((start, c))
                start = c
        out.append((start, a1))
    return out


def pieces(S: NDNode, g: int, w: int = 2):
    """Boxes (lo, hi) of the interfaces of separator S at granularity g."""
    lo, hi = S.sep_box(w)
    if S.is_leaf or g <= S.level:
        return [(lo, hi)]
    per_axis = []
    for b in range(3):
        iv = [(lo[b], hi[b])]
        if b != S.axis:
            for lam in range(S.level + 1, g + 1):
                iv = _refine(iv, _touching_cuts(S, lam, b, w))
        per_axis.append(iv)
    boxes = []
    for ix in per_axis[0]:
        for iy in per_axis[1]:
            for iz in per_axis[2]:
                boxes.append(((ix[0], iy[0], iz[0]), (ix[1], iy[1], iz[1])))
    return boxes


def box_cells(lo, hi, grid):
    """Cell indices of a box, ascending (x fastest)."""
    nx, ny = grid[0], grid[1]
    out = []
    for z in range(lo[2], hi[2]):
        for y in range(lo[1], hi[1]):
            for x in range(lo[0], hi[0]):
                out.append(x + nx * (y + ny * z))
    return out


def corner_cell(lo, grid):
    return lo[0] + grid[0] * (lo[1] + grid[1] * lo[2])


def finest_granularity(S: NDNode, depth: int) -> int:
    return S.level if S.is_leaf else max(S.level, depth - 1)
