"""spaQR for tall sparse least squares: plain FP64 oracle (test infrastructure).

Follows Algorithm 1 of the paper (Section 2.7) step by step:

* column scaling to unit 2-norm (Section 2.7, "the 2-norm of each column is
  a constant"; the constant is taken to be 1);
* geometric nested dissection with interfaces (Section 2.2, ``oracle.nd``);
* row matching + max-norm assignment of the unmatched rows (Section 2.2);
* per level m = d .. 1:
    - block Householder elimination of every level-m cluster s; R_s goes to
      W; the rows below the diagonal are compressed by a rank-revealing QR
      (truncated by the rank rule on sparsified levels, exact on the others)
      and reassigned to the neighbour cluster holding most of their squared
      norm (P_s, Sections 2.3 and 4.2);
    - on sparsified levels: interface scaling A_pp = U_pp [R_pp; 0]
      (Section 2.4), sparsification step 1 (rank-revealing QR of the rows
      below the scaled diagonal, Section 2.5.1) on every interface, then
      step 2 (rank-revealing QR of [A_np^T  A_p1n], Section 2.5.2);
    - merge of the interfaces one level up the cluster hierarchy
      (Section 2.6).

Data model.  A *cluster* is a live block of columns with an ordered list of
column "slots" (positions 0..N-1; a cluster's coarse columns reuse the first
slots of its list after sparsification).  Rows are held in *groups*: a group
is a dense block of rows owned by one cluster, stored over an explicit list
of slots, with the structural set of clusters its rows touch.

Readings where the paper is silent are listed in the module functions that
implement them (order of fronts and of step 2, row order inside fronts,
tie-breaks).  See ``factorize``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sl

from . import dense, graph_nd, nd

UNIT_ROUNDOFF = np.finfo(np.float64).eps / 2


class SpaqrError(RuntimeError):
    pass


@dataclass(eq=False)
class Cluster:
    key: tuple
    sep: nd.NDNode
    gran: int
    lo: tuple
    hi: tuple
    parent: "Cluster | None" = None
    children: list = field(default_factory=list)
    slots: list = field(default_factory=list)
    groups: list = field(default_factory=list)
    alive: bool = False

    def __repr__(self):
        return f"C{self.key}"


@dataclass(eq=False)
class Group:
    owner: Cluster
    data: np.ndarray
    slots: np.ndarray
    clus: set
    role: str = ""

    @property
    def nrows(self):
        return self.data.shape[0]

    def cols_of(self, slots, required=True):
        pos = {int(s): i for i, s in enumerate(self.slots)}
        idx = np.array([pos.get(int(s), -1) for s in slots], dtype=np.int64)
        if required and (idx < 0).any():
            raise SpaqrError("group lacks a column of a touched cluster")
        return idx


def _key(c):
    return c.key


def qr_flops(m, n):
    """Flops of an unpivoted Householder QR of an m x n matrix."""
    if m >= n:
        return 2.0 * m * n * n - 2.0 * n ** 3 / 3
    return 2.0 * n * m * m - 2.0 * m ** 3 / 3


# --------------------------------------------------------------------------
# analyze
# --------------------------------------------------------------------------

@dataclass
class Analysis:
    M: int
    N: int
    grid: tuple
    depth: int
    w: int
    nodes: list
    D: np.ndarray            # column norms of A
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray         # A (unscaled)
    ahat: np.ndarray         # values of A D^-1
    col_cluster: list        # finest cluster of each column
    row_owner: np.ndarray    # owner cluster index (into finest list) per row
    finest: list             # finest clusters sorted by key
    col_perm: np.ndarray     # columns in cluster order (finest clusters by key, slots ascending)


def _ancestor_or_self(a: nd.NDNode, b: nd.NDNode) -> bool:
    if b.level < a.level:
        return False
    return (b.path >> (b.level - a.level)) == a.path


def _graph_clusters(prob, depth):
    """Tree, clusters and matching for a matrix without a grid (readings G1-G3
    of oracle.graph_nd)."""
    adj_ptr, adj_idx = graph_nd.column_graph(prob.M, prob.N, np.asarray(prob.row_ptr), np.asarray(prob.col_idx))
    try:
        nodes = graph_nd.build_tree(prob.N, adj_ptr, adj_idx, depth)
    except ValueError as e:
        raise SpaqrError(str(e))
    for S in nodes:
        sets = graph_nd.piece_sets(S, depth, adj_ptr, adj_idx, prob.N)
        S.pieces = {}
        for g, lst in sets.items():
            S.pieces[g] = [Cluster(key=(S.rank, cols[0]), sep=S, gran=g, lo=None, hi=None, slots=list(cols))
                           for cols in lst]
        for g in range(S.level, max(sets)):
            where = {j: P for P in S.pieces[g] for j in P.slots}
            for c in S.pieces[g + 1]:
                par = {id(where[j]) for j in c.slots}
                if len(par) != 1:
                    raise SpaqrError("interface hierarchy does not nest")
                c.parent = where[c.slots[0]]
                c.parent.children.append(c)
        S.finest = S.pieces[max(sets)]
    try:
        match = graph_nd.max_product_matching(prob.M, prob.N, np.asarray(prob.row_ptr), np.asarray(prob.col_idx),
                                              np.asarray(prob.vals))
    except ValueError as e:
        raise SpaqrError(str(e))
    return nodes, match


def analyze(prob, depth: int, w: int = 2) -> Analysis:
    """Ordering, interfaces, hierarchy and row ownership (Section 2.2).

    With a cell grid the partition is geometric (oracle.nd); without one
    (prob.grid None) it is the graph nested dissection of oracle.graph_nd,
    with the max-product row matching."""
    M, N = prob.M, prob.N
    if M < N:
        raise SpaqrError("M < N")
    if getattr(prob, "grid", None) is None:
        return _analyze_general(prob, depth)
    grid = tuple(prob.grid) + (1,) * (3 - len(prob.grid))
    nodes = nd.build_tree(grid, depth, w)
    # clusters for every separator at every granularity it takes
    for S in nodes:
        S.pieces = {}
        gmax = nd.finest_granularity(S, depth)
        for g in range(S.level, gmax + 1):
            S.pieces[g] = []
            for lo, hi in nd.pieces(S, g, w):
                c = Cluster(key=(S.rank, nd.corner_cell(lo, grid)), sep=S, gran=g, lo=lo, hi=hi)
                S.pieces[g].append(c)
            S.pieces[g].sort(key=_key)
        for g in range(S.level, gmax):
            for c in S.pieces[g + 1]:
                par = [P for P in S.pieces[g]
                       if all(P.lo[a] <= c.lo[a] and c.hi[a] <= P.hi[a] for a in range(3))]
                if len(par) != 1:
                    raise SpaqrError("interface hierarchy does not nest")
                c.parent = par[0]
                par[0].children.append(c)
        S.finest = S.pieces[gmax]
    finest = sorted([c for S in nodes for c in S.finest], key=_key)
    col_cluster = [None] * N
    for ci, c in enumerate(finest):
        c.slots = nd.box_cells(c.lo, c.hi, grid)
        c.index = ci
        for j in c.slots:
            if col_cluster[j] is not None:
                raise SpaqrError("cell in two clusters")
            col_cluster[j] = c
    if any(c is None for c in col_cluster):
        raise SpaqrError("cell in no cluster")

    match = np.arange(N, dtype=np.int64)   # column j <-> its Laplacian row j (reading R3)
    return _finish(prob, depth, w, grid, nodes, finest, col_cluster, match)


def _analyze_general(prob, depth):
    M, N = prob.M, prob.N
    nodes, match = _graph_clusters(prob, depth)
    finest = sorted([c for S in nodes for c in S.finest], key=_key)
    col_cluster = [None] * N
    for ci, c in enumerate(finest):
        c.index = ci
        for j in c.slots:
            if col_cluster[j] is not None:
                raise SpaqrError("column in two clusters")
            col_cluster[j] = c
    if any(c is None for c in col_cluster):
        raise SpaqrError("column in no cluster")
    return _finish(prob, depth, 0, None, nodes, finest, col_cluster, match)


def _finish(prob, depth, w, grid, nodes, finest, col_cluster, match):
    M, N = prob.M, prob.N
    # column scaling (Section 2.7)
    row_ptr = np.asarray(prob.row_ptr, dtype=np.int64)
    col_idx = np.asarray(prob.col_idx, dtype=np.int64)
    vals = np.asarray(prob.vals, dtype=np.float64)
    D = np.sqrt(np.bincount(col_idx, weights=vals * vals, minlength=N))
    if (D == 0).any():
        raise SpaqrError("empty column")
    ahat = vals / D[col_idx]

    # no row may touch two sibling subtrees
    for r in range(M):
        cs = col_idx[row_ptr[r]:row_ptr[r + 1]]
        ns = {col_cluster[j].sep for j in cs}
        ns = list(ns)
        for i in range(len(ns)):
            for k in range(i + 1, len(ns)):
                if not (_ancestor_or_self(ns[i], ns[k]) or _ancestor_or_self(ns[k], ns[i])):
                    raise SpaqrError(f"row {r} touches two sibling subtrees")

    # row ownership (Section 2.2): the row matched to column j goes to j's
    # cluster; every other row goes to the finest cluster holding the
    # largest sum of its squared (scaled) entries, ties to the lowest id
    owner = np.full(M, -1, dtype=np.int64)
    owner[match] = [col_cluster[j].index for j in range(N)]
    for r in range(M):
        if owner[r] >= 0:
            continue
        lo, hi = row_ptr[r], row_ptr[r + 1]
        acc = {}
        for j, v in zip(col_idx[lo:hi], ahat[lo:hi]):
            ci = col_cluster[j].index
            acc[ci] = acc.get(ci, 0.0) + v * v
        best = max(acc.items(), key=lambda kv: (kv[1], -kv[0]))
        owner[r] = best[0]
    col_perm = np.array([j for c in finest for j in c.slots], dtype=np.int64)
    return Analysis(M=M, N=N, grid=grid, depth=depth, w=w, nodes=nodes, D=D, row_ptr=row_ptr,
                    col_idx=col_idx, vals=vals, ahat=ahat, col_cluster=col_cluster, row_owner=owner,
                    finest=finest, col_perm=col_perm)


def initial_groups(an: Analysis):
    """Rows of every finest cluster, grouped by the set of clusters they touch.

    Inside an owner, rows are in ascending original index; groups are ordered
    by their first row.
    """
    groups = {c.index: [] for c in an.finest}
    sig_rows = {}
    for r in range(an.M):
        lo, hi = an.row_ptr[r], an.row_ptr[r + 1]
        sig = frozenset(an.col_cluster[j].index for j in an.col_idx[lo:hi])
        sig_rows.setdefault((int(an.row_owner[r]), sig), []).append(r)
    order = sorted(sig_rows.items(), key=lambda kv: kv[1][0])
    for (oi, sig), rows in order:
        clus = sorted((an.finest[i] for i in sig), key=_key)
        slots = np.array([s for c in clus for s in c.slots], dtype=np.int64)
        pos = {int(s): i for i, s in enumerate(slots)}
        data = np.zeros((len(rows), len(slots)))
        for i, r in enumerate(rows):
            lo, hi = an.row_ptr[r], an.row_ptr[r + 1]
            for j, v in zip(an.col_idx[lo:hi], an.ahat[lo:hi]):
                data[i, pos[int(j)]] = v
        groups[oi].append(Group(owner=an.finest[oi], data=data, slots=slots, clus=set(clus)))
    return groups


# --------------------------------------------------------------------------
# factorization
# --------------------------------------------------------------------------

@dataclass
class Factor:
    an: Analysis
    eps: float
    ops: list                 # W as a list of elementary ops, creation order
    ranks: list               # every rank decision, in decision order
    stats: dict
    ledger: dict


def _gather(groups, clusters):
    cols = (np.concatenate([np.asarray(c.slots, dtype=np.int64) for c in clusters])
            if clusters else np.zeros(0, dtype=np.int64))
    F = np.zeros((sum(g.nrows for g in groups), cols.shape[0]))
    r0 = 0
    for g in groups:
        idx = g.cols_of(cols, required=False)
        m = idx >= 0
        F[r0:r0 + g.nrows, m] = g.data[:, idx[m]]
        r0 += g.nrows
    return F, cols


class _State:
    def __init__(self, an: Analysis, eps: float, skip: int, forced):
        self.an = an
        self.eps = eps
        self.skip = skip
        self.forced = list(forced) if forced is not None else None
        self.live = set()
        self.ops = []
        self.ranks = []
        self.ledger = {k: [0.0, 0.0] for k in ("eliminate", "reassign", "scale", "sparsify", "merge")}
        self.stats = dict(aspect=[], ranks_step1=[], ranks_step2=[], rounds_elim=[], rounds_step2=[],
                          top_separator=None)
        self.level = 0
        self.log = None           # per rank-revealing QR records, when asked for (tests)

    # ---- helpers -------------------------------------------------------
    def sorted_live(self):
        return sorted(self.live, key=_key)

    def all_groups(self):
        for c in self.sorted_live():
            yield from c.groups

    def next_rank(self, rule_rank):
        if self.forced is None:
            return None
        if not self.forced:
            raise SpaqrError("forced rank list exhausted")
        return self.forced.pop(0)

    def sparsified(self, level):
        """Levels that are scaled and sparsified (Section 4: the first
        leaf-side levels are skipped; the root has no interfaces left)."""
        return 2 <= level <= self.an.depth - self.skip

    def pivoted(self, C, kind, eps=None):
        eps = self.eps if eps is None else eps
        forced = self.next_rank(None)
        if forced is None:
            r, rows, perm, V, tau = dense.pivoted_qr(C, eps)
        else:
            r, rows, perm, V, tau = dense.pivoted_qr(C, 0.0)
            r = min(forced, r)
            rows, V, tau = rows[:r], V[:, :r], tau[:r]
            # rows beyond the forced rank must also be dropped from Q^T C
        self.ranks.append(r)
        m, n = C.shape
        if self.log is not None:
            self.log.append(dict(kind=kind, level=self.level, eps=eps, m=m, n=n, rank=r, rows=rows.copy(),
                                 perm=perm.copy(), normf2=float(np.sum(C * C)),
                                 forced=forced is not None))
        phase = "reassign" if kind == "reassign" else "sparsify"
        self.ledger[phase][0] += 4 * m * n * r - 2 * r * r * (m + n) + 4 * r ** 3 / 3 + 2 * m * n
        self.ledger[phase][1] += 8 * (m * n + r * n)
        return r, rows, V, tau

    # ---- front of an eliminated cluster ----------------------------------
    def front_groups(self, s):
        owned = list(s.groups)
        foreign = []
        for c in self.sorted_live():
            if c is s:
                continue
            for g in c.groups:
                if s in g.clus:
                    foreign.append(g)
        return owned, foreign

    def neighbours(self, s):
        owned, foreign = self.front_groups(s)
        nb = set()
        for g in owned + foreign:
            nb |= g.clus
        nb.discard(s)
        return nb

    def reassign_rows(self, rows, slots, clus, col_ranges, source):
        """Give each row to the cluster holding most of its squared norm."""
        out = {}
        for i in range(rows.shape[0]):
            best, bestv = None, -1.0
            for c, (a, b) in zip(clus, col_ranges):
                v = float(np.dot(rows[i, a:b], rows[i, a:b]))
                if v > bestv:
                    best, bestv = c, v
            out.setdefault(best, []).append(i)
        for c in sorted(out, key=_key):
            c.groups.append(Group(owner=c, data=rows[out[c]].copy(), slots=slots.copy(), clus=set(clus)))

    def eliminate(self, s):
        owned, foreign = self.front_groups(s)
        nb = set()
        for g in owned + foreign:
            nb |= g.clus
        nb.discard(s)
        N_s = sorted(nb, key=_key)
        F, cols = _gather(owned + foreign, [s] + N_s)
        c_s = len(s.slots)
        r_s = sum(g.nrows for g in owned)
        if r_s < c_s:
            raise SpaqrError(f"cluster {s.key} has fewer rows ({r_s}) than columns ({c_s})")
        m, n = F.shape
        c_N = n - c_s
        dense.householder_qr(F, c_s)
        self.ledger["eliminate"][0] += 2 * m * c_s ** 2 - 2 * c_s ** 3 / 3 + 4 * m * c_s * c_N - 2 * c_s ** 2 * c_N
        self.ledger["eliminate"][1] += 8 * (2 * m * n)
        R = np.triu(F[:c_s, :]).copy()
        self.ops.append(("elim", np.array(s.slots), cols[c_s:].copy(), R))
        # rows of other owners stay with their owner, now over the neighbour columns
        r0 = r_s
        nslots = cols[c_s:].copy()
        for g in foreign:
            g.data = F[r0:r0 + g.nrows, c_s:].copy()
            g.slots = nslots.copy()
            g.clus = set(N_s)
            g.role = ""
            r0 += g.nrows
        # rows below the diagonal: compressed, then reassigned (P_s).  On a
        # sparsified level they are sparsified like the interfaces (the
        # reassign phase of Section 4.2); on the skipped leaf-side levels
        # nothing is sparsified, so the compression is exact: the
        # rank-revealing QR stops only at the numerical rank.
        if c_N > 0 and r_s > c_s:
            E = F[c_s:r_s, c_s:]
            eps_r = self.eps if self.sparsified(self.level) else 0.0
            r, RE, V, tau = self.pivoted(E, "reassign", eps_r)
            ranges = []
            a = 0
            for c in N_s:
                ranges.append((a, a + len(c.slots)))
                a += len(c.slots)
            if r:
                self.reassign_rows(RE, nslots, N_s, ranges, s)
        s.groups = []
        s.alive = False
        self.live.discard(s)

    # ---- interface scaling (Section 2.4) --------------------------------
    def scale_all(self, level):
        ifaces = self.sorted_live()
        Rpp = {}
        aspects = []
        for p in ifaces:
            groups = p.groups
            nb = set()
            for g in groups:
                nb |= g.clus
            nb.discard(p)
            others = sorted(nb, key=_key)
            F, cols = _gather(groups, [p] + others)
            m, n = F.shape
            c_p = len(p.slots)
            if m < c_p:
                raise SpaqrError(f"interface {p.key} has fewer rows than columns")
            aspects.append(m / c_p)
            normf = float(np.linalg.norm(F[:, :c_p]))
            dense.householder_qr(F, c_p)
            self.ledger["scale"][0] += 2 * m * c_p ** 2 - 2 * c_p ** 3 / 3 + 4 * m * c_p * (n - c_p) - 2 * c_p ** 2 * (n - c_p)
            self.ledger["scale"][1] += 8 * 2 * m * n
            R = np.triu(F[:c_p, :c_p]).copy()
            if np.min(np.abs(np.diag(R))) <= 64 * UNIT_ROUNDOFF * normf:
                raise SpaqrError(f"interface {p.key} is rank deficient")
            self.ops.append(("scale", np.array(p.slots), R))
            Rpp[p] = R
            p1data = F[:c_p, :].copy()
            p1data[:, :c_p] = np.eye(c_p)
            newg = [Group(owner=p, data=p1data, slots=cols.copy(), clus={p} | set(others), role="p1")]
            if m > c_p and n > c_p:
                newg.append(Group(owner=p, data=F[c_p:, c_p:].copy(), slots=cols[c_p:].copy(),
                                  clus=set(others), role="p2"))
            p.groups = newg
        # right scaling of every column block: B[q][p] <- B[q][p] R_pp^-1
        for g in self.all_groups():
            for q in sorted(g.clus, key=_key):
                if g.role == "p1" and g.owner is q:
                    continue
                idx = g.cols_of(q.slots)
                B = g.data[:, idx]
                g.data[:, idx] = sl.solve_triangular(Rpp[q], B.T, trans="T", lower=False).T
                self.ledger["scale"][0] += g.nrows * len(q.slots) ** 2
                self.ledger["scale"][1] += 8 * 2 * g.nrows * len(q.slots)
        if aspects:
            self.stats["aspect"].append((level, float(np.median(aspects))))

    # ---- sparsification step 1 (Section 2.5.1) --------------------------
    def step1_all(self, level):
        rk = []
        for p in self.sorted_live():
            p2 = [g for g in p.groups if g.role == "p2"]
            if not p2:
                continue
            g = p2[0]
            r, rows, V, tau = self.pivoted(g.data, "step1")
            rk.append(r)
            if r == 0:
                p.groups.remove(g)
            else:
                g.data = rows
        self.stats["ranks_step1"].append((level, rk))

    # ---- sparsification step 2 (Section 2.5.2) --------------------------
    @staticmethod
    def p1_of(p):
        for g in p.groups:
            if g.role == "p1":
                return g
        raise SpaqrError("interface without scaled rows")

    def conflict(self, p, q):
        return q in self.p1_of(p).clus or p in self.p1_of(q).clus

    def step2(self, p, level):
        p1 = self.p1_of(p)
        blocks = [g for g in self.all_groups() if g is not p1 and p in g.clus]
        others = sorted(p1.clus - {p}, key=_key)
        oslots = (np.concatenate([np.asarray(c.slots, dtype=np.int64) for c in others])
                  if others else np.zeros(0, dtype=np.int64))
        parts = [g.data[:, g.cols_of(p.slots)].T for g in blocks]
        parts.append(p1.data[:, p1.cols_of(oslots)])
        C = np.hstack(parts) if parts else np.zeros((len(p.slots), 0))
        r, rows, V, tau = self.pivoted(C, "step2")
        self.stats["_rk2"].append(r)
        self.ops.append(("sparsify", np.array(p.slots), V, tau))
        off = 0
        keep = p.slots[:r]
        for g in blocks:
            g.data[:, g.cols_of(keep)] = rows[:, off:off + g.nrows].T
            off += g.nrows
        p1.data[:r, p1.cols_of(oslots)] = rows[:, off:]
        p1.data[:r, p1.cols_of(keep)] = np.eye(r)
        p1.data = p1.data[:r].copy()
        p.slots = list(keep)
        if r == 0:
            self.vanish(p)

    def vanish(self, p):
        """An interface with no coarse column left: its remaining rows move on."""
        p.alive = False
        self.live.discard(p)
        for g in self.all_groups():
            g.clus.discard(p)
        for g in p.groups:
            if g.role == "p1" or g.nrows == 0:
                continue
            g.clus.discard(p)
            clus = sorted(g.clus, key=_key)
            if not clus:
                continue
            ranges = []
            for c in clus:
                idx = g.cols_of(c.slots)
                ranges.append(idx)
            # reorder the row's columns cluster by cluster for the norm test
            cols = np.concatenate(ranges)
            rows = g.data[:, cols]
            slots = g.slots[cols]
            rr, a = [], 0
            for idx in ranges:
                rr.append((a, a + len(idx)))
                a += len(idx)
            self.reassign_rows(rows, slots, clus, rr, p)
        p.groups = []

    # ---- merge (Section 2.6) ---------------------------------------------
    def merge(self, level):
        an = self.an
        for S in an.nodes:
            if S.level >= level or S.is_leaf:
                continue
            fin = nd.finest_granularity(S, an.depth)
            cur = min(max(S.level, level - 1), fin)
            tgt = min(max(S.level, level - 2), fin)
            if tgt >= cur:
                continue
            for P in S.pieces[tgt]:
                kids = sorted([c for c in P.children if c.alive], key=_key)
                P.slots = [j for c in kids for j in c.slots]
                P.groups = [g for c in kids for g in c.groups]
                for g in P.groups:
                    g.owner = P
                kidset = set(kids)
                for c in kids:
                    c.alive = False
                    c.groups = []
                    self.live.discard(c)
                P.alive = len(P.slots) > 0
                if P.alive:
                    self.live.add(P)
                for g in self.all_groups():
                    if g.clus & kidset:
                        g.clus -= kidset
                        if P.alive:
                            g.clus.add(P)


def _select_round(pending, conflict):
    sel = []
    for p in pending:
        if all(not conflict(p, q) for q in sel):
            sel.append(p)
    return sel


def factorize(an: Analysis, eps: float, skip: int, forced_ranks=None, log=None) -> Factor:
    """Run Algorithm 1.

    Readings (the paper leaves these open):

    * sparsified levels are m with 2 <= m <= d - skip (Section 4: the first
      leaf-side levels are not sparsified);
    * a front holds the eliminated cluster's own rows (its groups in order),
      then the rows of other owners that touch it, by owner id then group
      order; its columns are the cluster's, then every neighbour cluster's
      in id order;
    * clusters of one level are eliminated in rounds: each round takes, in
      id order, every pending cluster that shares no front row and no front
      column with a cluster already taken in the round; likewise step 2 runs
      in rounds with p ~ q when q is among the columns of p's scaled rows or
      p among q's.  Inside a round the order does not change the result;
    * rows below the diagonal of an eliminated cluster are compressed by a
      column-pivoted QR that keeps the leading rows of Q^T E, and each kept
      row goes to the neighbour cluster with the largest sum of its squared
      entries (ties to the lowest id).  On sparsified levels the rank rule
      of Section 4 truncates it (Section 4.2 names the sparsification of
      these rows as part of the reassign phase); on the leaf-side levels
      where sparsification is skipped the compression is exact.  Every
      rank-revealing QR also stops at the numerical rank
      (|R_ii| <= 1000 u ||C||_F), where an unpivoted or further-pivoted QR
      would be steered by rounding error;
    * scaling is applied to all interfaces of the level: every left
      transform U_pp^T first, then every right transform R_pp^-1;
    * step 2 compresses the column block of p over every row except p's
      own scaled rows, next to those scaled rows over the other columns.
    """
    st = _State(an, eps, skip, forced_ranks)
    st.log = log
    st.stats["_rk2"] = []
    groups = initial_groups(an)
    for c in an.finest:
        c.groups = groups[c.index]
        c.alive = True
        st.live.add(c)
    d = an.depth
    for m in range(d, 0, -1):
        st.level = m
        pending = sorted([c for c in st.live if c.sep.level == m], key=_key)
        if m == 1 and pending:
            st.stats["top_separator"] = (len(pending[0].slots), sum(g.nrows for g in pending[0].groups))
        nrounds = 0
        while pending:
            nbs = {s: st.neighbours(s) for s in pending}
            sel = _select_round(pending, lambda a, b: b in nbs[a] or a in nbs[b])
            for s in sel:
                st.eliminate(s)
            pending = [s for s in pending if s not in sel]
            nrounds += 1
        st.stats["rounds_elim"].append((m, nrounds))
        if st.sparsified(m) and st.live:
            st.scale_all(m)
            st.step1_all(m)
            pending = st.sorted_live()
            st.stats["_rk2"] = []
            nrounds = 0
            while pending:
                sel = _select_round(pending, st.conflict)
                for p in sel:
                    st.step2(p, m)
                pending = [p for p in pending if p not in sel]
                nrounds += 1
            st.stats["ranks_step2"].append((m, list(st.stats["_rk2"])))
            st.stats["rounds_step2"].append((m, nrounds))
        st.merge(m)
    if st.live:
        raise SpaqrError("clusters left after the root level")
    if st.forced:
        raise SpaqrError("forced rank list not fully used")
    st.stats.pop("_rk2", None)
    memf = 0
    for op in st.ops:
        if op[0] == "elim":
            cs = op[1].shape[0]
            memf += cs * (cs + 1) // 2 + cs * op[2].shape[0]
        elif op[0] == "scale":
            cp = op[1].shape[0]
            memf += cp * (cp + 1) // 2
        else:
            memf += op[2].shape[0] * op[2].shape[1]
    st.stats["memF"] = memf
    return Factor(an=an, eps=eps, ops=st.ops, ranks=st.ranks, stats=st.stats,
                  ledger={k: tuple(v) for k, v in st.ledger.items()})
