"""Nested dissection, interfaces and row matching for matrices given
without a cell grid (oracle, test infrastructure only).

Restates Section 2.2 (partitioning of G(A^T A) into a nested-dissection
tree, interfaces of every separator at every granularity, a row matching
with large entries and max-norm assignment of the other rows; the paper
uses a hypergraph partitioner and the MC64 matching) with these readings:

* G1 (partitioning): G is the column graph of A^T A (columns i != j
  adjacent when a row holds both).  A region V at tree level < d is split
  by a level structure: a breadth-first search over G[V] from the lowest
  column of V (neighbours taken in ascending order; when the queue runs
  dry the lowest unvisited column starts again at level 0), then a second
  search from the lowest column on the deepest level of the first; the
  separator is the first level k whose cumulative count reaches half of
  |V| (2 * sum_{l <= k} >= |V|), the low child the levels below it, the
  high child the levels above.  Adjacent columns differ by at most one
  level, so no column of one child is adjacent to the other: no row
  touches two sibling subtrees.  Both children must be non-empty.
* G2 (interfaces): a separator S of level l is one interface at
  granularity l; at granularity g+1 every interface P of granularity g is
  split into the connected components (in G[P]) of its columns adjacent to
  a separator column of a level-(g+1) descendant of S, and those of its
  other columns.  Pieces of g+1 therefore nest in those of g (the analogue
  of cutting the separator's face by the descendants' cut planes in the
  geometric form).  Pieces are ordered by their lowest column.
* G3 (matching): the column-to-row matching maximising the product of
  |a_ij| (MC64's objective): minimum total cost with c_ij = log(max_k |a_kj|)
  - log |a_ij| over matchings that cover every column; unique when the
  values are in general position.  A matched row goes to its column's
  finest cluster; every other row to the finest cluster holding the
  largest sum of its squared scaled entries (ties to the lowest id).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import min_weight_full_bipartite_matching


@dataclass(eq=False)
class GNode:
    level: int
    path: int
    region: np.ndarray                 # every column of the subtree, ascending
    sep_cols: np.ndarray = None        # the node's own columns (separator, or the leaf)
    children: list = field(default_factory=list)
    parent: "GNode | None" = None
    rank: int = -1

    @property
    def is_leaf(self) -> bool:
        return not self.children

    def subtree(self):
        out = [self]
        for c in self.children:
            out.extend(c.subtree())
        return out


def column_graph(M, N, row_ptr, col_idx):
    """Adjacency of G(A^T A) without the diagonal, as a CSR pattern."""
    rows = np.repeat(np.arange(M), np.diff(row_ptr))
    A = sp.csr_matrix((np.ones(len(col_idx)), (rows, np.asarray(col_idx))), shape=(M, N))
    G = (A.T @ A).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    return G.indptr, G.indices


def _levels(V, start, adj_ptr, adj_idx, inV):
    """Breadth-first level of every column of V (forest over G[V])."""
    lev = {}
    order = [int(start)]
    lev[int(start)] = 0
    head = 0
    rest = iter(V)
    while True:
        while head < len(order):
            v = order[head]
            head += 1
            for u in adj_idx[adj_ptr[v]:adj_ptr[v + 1]]:
                u = int(u)
                if inV[u] and u not in lev:
                    lev[u] = lev[v] + 1
                    order.append(u)
        nxt = None
        for u in rest:
            if int(u) not in lev:
                nxt = int(u)
                break
        if nxt is None:
            return lev
        lev[nxt] = 0
        order.append(nxt)


def bisect(V, adj_ptr, adj_idx, N):
    inV = np.zeros(N, dtype=bool)
    inV[V] = True
    lev = _levels(V, V[0], adj_ptr, adj_idx, inV)
    deepest = max(lev.values())
    r1 = min(v for v, l in lev.items() if l == deepest)
    lev = _levels(V, r1, adj_ptr, adj_idx, inV)
    L = max(lev.values())
    cnt = np.bincount(np.array(list(lev.values())), minlength=L + 1)
    cum = np.cumsum(cnt)
    k = int(np.argmax(2 * cum >= len(V)))
    low = np.array(sorted(v for v, l in lev.items() if l < k), dtype=np.int64)
    sep = np.array(sorted(v for v, l in lev.items() if l == k), dtype=np.int64)
    high = np.array(sorted(v for v, l in lev.items() if l > k), dtype=np.int64)
    return low, sep, high


def build_tree(N, adj_ptr, adj_idx, depth):
    def rec(region, level, path, parent):
        node = GNode(level=level, path=path, region=region, parent=parent)
        if level < depth:
            low, sep, high = bisect(region, adj_ptr, adj_idx, N)
            if len(low) == 0 or len(high) == 0:
                raise ValueError(f"graph too small to split at level {level}")
            node.sep_cols = sep
            node.children = [rec(low, level + 1, 2 * path, node), rec(high, level + 1, 2 * path + 1, node)]
        else:
            node.sep_cols = region
        return node

    root = rec(np.arange(N, dtype=np.int64), 1, 0, None)
    nodes = root.subtree()
    nodes.sort(key=lambda n: (-n.level, n.path))
    for i, n in enumerate(nodes):
        n.rank = i
    return nodes


def _components(cols, adj_ptr, adj_idx, N):
    """Connected components of G[cols], each ascending, ordered by lowest column."""
    inset = np.zeros(N, dtype=bool)
    inset[cols] = True
    seen = set()
    comps = []
    for s in sorted(int(c) for c in cols):
        if s in seen:
            continue
        comp = [s]
        seen.add(s)
        head = 0
        while head < len(comp):
            v = comp[head]
            head += 1
            for u in adj_idx[adj_ptr[v]:adj_ptr[v + 1]]:
                u = int(u)
                if inset[u] and u not in seen:
                    seen.add(u)
                    comp.append(u)
        comps.append(sorted(comp))
    comps.sort(key=lambda c: c[0])
    return comps


def piece_sets(S: GNode, depth, adj_ptr, adj_idx, N):
    """{granularity: [sorted column lists]} for separator S (reading G2)."""
    gmax = S.level if S.is_leaf else max(S.level, depth - 1)
    out = {S.level: [sorted(int(c) for c in S.sep_cols)]}
    sub = S.subtree()
    for g in range(S.level, gmax):
        tcols = np.zeros(N, dtype=bool)
        for T in sub:
            if T.level == g + 1 and not T.is_leaf:
                tcols[T.sep_cols] = True
        cut = np.zeros(N, dtype=bool)
        for v in S.sep_cols:
            nb = adj_idx[adj_ptr[v]:adj_ptr[v + 1]]
            cut[v] = bool(tcols[nb].any())
        nxt = []
        for P in out[g]:
            P = np.asarray(P, dtype=np.int64)
            a = P[cut[P]]
            b = P[~cut[P]]
            nxt.extend(_components(a, adj_ptr, adj_idx, N) if len(a) else [])
            nxt.extend(_components(b, adj_ptr, adj_idx, N) if len(b) else [])
        nxt.sort(key=lambda c: c[0])
        out[g + 1] = nxt
    return out


def max_product_matching(M, N, row_ptr, col_idx, vals):
    """Row matched to each column (reading G3)."""
    rows = np.repeat(np.arange(M), np.diff(row_ptr))
    a = np.abs(np.asarray(vals, dtype=np.float64))
    if (a == 0).any():
        raise ValueError("explicit zero entries")
    colmax = np.zeros(N)
    np.maximum.at(colmax, col_idx, a)
    cost = np.log(colmax[col_idx]) - np.log(a)
    # every matching that covers the columns has N edges, so a constant
    # offset keeps the optimum and keeps every weight strictly positive
    B = sp.csr_matrix((cost + 1.0, (np.asarray(col_idx), rows)), shape=(N, M))
    r, c = min_weight_full_bipartite_matching(B)
    match = np.full(N, -1, dtype=np.int64)
    match[r] = c
    if (match < 0).any():
        raise ValueError("no matching covers every column")
    return match
