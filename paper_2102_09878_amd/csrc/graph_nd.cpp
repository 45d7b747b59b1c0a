// Analysis of matrices handed over without a cell grid (Section 2.2 with
// the hypergraph partitioner and the MC64 matching replaced by the rules
// below).  Host code.
//
// Partitioning: G is the column graph of A^T A (two columns adjacent when a
// row holds both).  A region at tree level < d is split by a breadth-first
// level structure over the region: a first search from its lowest column
// (neighbours in ascending order; when the queue runs dry the lowest
// unvisited column restarts at level 0), a second from the lowest column of
// the first search's deepest level.  The separator is the first level whose
// cumulative count reaches half the region, the low child the levels below,
// the high child the levels above; adjacent columns are at most one level
// apart, so no row reaches both children.
//
// Interfaces: a separator of level l is one interface at granularity l; at
// granularity g+1 each interface of granularity g splits into the connected
// components (within the interface) of its columns adjacent to a separator
// column of a level-(g+1) descendant, and of its other columns.  Pieces
// are ordered by their lowest column, so the keys are (separator rank,
// lowest column) and pieces of g+1 nest in those of g.
//
// Matching: the column-to-row assignment of largest product of |a_ij|, as
// a minimum-cost assignment with c_ij = log max_k |a_kj| - log |a_ij| >= 0,
// solved by shortest augmenting paths (Dijkstra over reduced costs kept
// non-negative by row and column potentials).
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <queue>

#include "spaqr_impl.h"

namespace spaqr {

namespace {

struct Graph {
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;  // ascending per column
};

Graph column_graph(const Plan& P) {
  // A^T pattern first (rows of each column)
  std::vector<int64_t> cptr(P.N + 1, 0);
  for (int64_t e = 0; e < P.nnz; ++e) cptr[P.col_idx[e] + 1]++;
  for (int64_t j = 0; j < P.N; ++j) cptr[j + 1] += cptr[j];
  std::vector<int64_t> crow(P.nnz);
  std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
  for (int64_t r = 0; r < P.M; ++r)
    for (int64_t e = P.row_ptr[r]; e < P.row_ptr[r + 1]; ++e) crow[fill[P.col_idx[e]]++] = r;
  Graph G;
  G.ptr.assign(P.N + 1, 0);
  std::vector<int64_t> mark(P.N, -1);
  std::vector<int32_t> nb;
  for (int64_t j = 0; j < P.N; ++j) {
    nb.clear();
    mark[j] = j;
    for (int64_t k = cptr[j]; k < cptr[j + 1]; ++k) {
      const int64_t r = crow[k];
      for (int64_t e = P.row_ptr[r]; e < P.row_ptr[r + 1]; ++e) {
        const int32_t c = P.col_idx[e];
        if (mark[c] != j) {
          mark[c] = j;
          nb.push_back(c);
        }
      }
    }
    std::sort(nb.begin(), nb.end());
    G.idx.insert(G.idx.end(), nb.begin(), nb.end());
    G.ptr[j + 1] = (int64_t)G.idx.size();
  }
  return G;
}

// Breadth-first levels over the region V (ascending), as described above.
// lev[v] is written for v in V (and -1 must hold for v in V on entry).
void levels(const Graph& G, const std::vector<int>& V, int start, const std::vector<char>& inV,
            std::vector<int>& lev, std::vector<int>& order) {
  order.clear();
  order.push_back(start);
  lev[start] = 0;
  size_t head = 0, rest = 0;
  for (;;) {
    while (head < order.size()) {
      const int v = order[head++];
      for (int64_t k = G.ptr[v]; k < G.ptr[v + 1]; ++k) {
        const int u = G.idx[k];
        if (inV[u] && lev[u] < 0) {
          lev[u] = lev[v] + 1;
          order.push_back(u);
        }
      }
    }
    while (rest < V.size() && lev[V[rest]] >= 0) ++rest;
    if (rest == V.size()) return;
    lev[V[rest]] = 0;
    order.push_back(V[rest]);
  }
}

struct GNodeTmp {
  int level;
  int64_t path;
  std::vector<int> region, sep;  // ascending
  int child[2] = {-1, -1};
  int parent = -1;
};

// Connected components of the columns `cols` (ascending) inside G,
// each ascending; appended to out.
void components(const Graph& G, const std::vector<int>& cols, std::vector<char>& in, std::vector<char>& seen,
                std::vector<std::vector<int>>& out) {
  for (int c : cols) in[c] = 1;
  std::vector<int> q;
  for (int s : cols) {
    if (seen[s]) continue;
    q.assign(1, s);
    seen[s] = 1;
    for (size_t h = 0; h < q.size(); ++h) {
      const int v = q[h];
      for (int64_t k = G.ptr[v]; k < G.ptr[v + 1]; ++k) {
        const int u = G.idx[k];
        if (in[u] && !seen[u]) {
          seen[u] = 1;
          q.push_back(u);
        }
      }
    }
    std::sort(q.begin(), q.end());
    out.push_back(q);
  }
  for (int c : cols) in[c] = 0, seen[c] = 0;
}

}  // namespace

void graph_partition(Plan& P) {
  const Graph G = column_graph(P);
  const int N = (int)P.N;
  std::vector<GNodeTmp> tmp;
  std::vector<char> inV(N, 0);
  std::vector<int> lev(N, -1), order;
  // explicit stack: (node index to fill)
  GNodeTmp root;
  root.level = 1;
  root.path = 0;
  root.region.resize(N);
  std::iota(root.region.begin(), root.region.end(), 0);
  tmp.push_back(std::move(root));
  std::vector<int> work{0};
  while (!work.empty()) {
    const int id = work.back();
    work.pop_back();
    if (tmp[id].level >= P.depth) {
      tmp[id].sep = tmp[id].region;
      continue;
    }
    const std::vector<int> V = tmp[id].region;
    for (int v : V) inV[v] = 1;
    levels(G, V, V[0], inV, lev, order);
    int deepest = 0;
    for (int v : V) deepest = std::max(deepest, lev[v]);
    int r1 = N;
    for (int v : V)
      if (lev[v] == deepest) r1 = std::min(r1, v);
    for (int v : V) lev[v] = -1;
    levels(G, V, r1, inV, lev, order);
    int L = 0;
    for (int v : V) L = std::max(L, lev[v]);
    std::vector<int64_t> cnt(L + 1, 0);
    for (int v : V) cnt[lev[v]]++;
    int k = 0;
    int64_t cum = 0;
    for (; k <= L; ++k) {
      cum += cnt[k];
      if (2 * cum >= (int64_t)V.size()) break;
    }
    GNodeTmp lo, hi;
    std::vector<int> sep;
    for (int v : V) {
      if (lev[v] < k)
        lo.region.push_back(v);
      else if (lev[v] == k)
        sep.push_back(v);
      else
        hi.region.push_back(v);
    }
    for (int v : V) inV[v] = 0, lev[v] = -1;
    if (lo.region.empty() || hi.region.empty())
      throw Error(SPAQR_EARG, "matrix graph too small for the requested nested-dissection depth");
    tmp[id].sep = sep;
    lo.level = hi.level = tmp[id].level + 1;
    lo.path = 2 * tmp[id].path;
    hi.path = 2 * tmp[id].path + 1;
    lo.parent = hi.parent = id;
    const int a = (int)tmp.size();
    tmp.push_back(std::move(lo));
    tmp.push_back(std::move(hi));
    tmp[id].child[0] = a;
    tmp[id].child[1] = a + 1;
    work.push_back(a + 1);
    work.push_back(a);
  }
  // elimination rank: leaves first, left to right, then up to the root
  std::vector<int> ord(tmp.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) {
    if (tmp[x].level != tmp[y].level) return tmp[x].level > tmp[y].level;
    return tmp[x].path < tmp[y].path;
  });
  std::vector<int> rank_of(tmp.size());
  for (size_t r = 0; r < ord.size(); ++r) rank_of[ord[r]] = (int)r;
  P.nodes.assign(tmp.size(), NDNode());
  for (size_t i = 0; i < tmp.size(); ++i) {
    NDNode& d = P.nodes[rank_of[i]];
    d.level = tmp[i].level;
    d.path = tmp[i].path;
    d.axis = tmp[i].child[0] >= 0 ? 0 : -1;
    d.parent = tmp[i].parent >= 0 ? rank_of[tmp[i].parent] : -1;
    for (int c = 0; c < 2; ++c) d.child[c] = tmp[i].child[c] >= 0 ? rank_of[tmp[i].child[c]] : -1;
    d.rank = rank_of[i];
  }
  // separator columns by rank
  std::vector<const std::vector<int>*> sep_of(tmp.size());
  for (size_t i = 0; i < tmp.size(); ++i) sep_of[rank_of[i]] = &tmp[i].sep;

  // interfaces of every separator at every granularity
  struct Piece {
    int64_t k0, k1;
    int sep, gran;
    std::vector<int> cols;
  };
  std::vector<Piece> pieces;
  std::vector<char> tcol(N, 0), in(N, 0), seen(N, 0);
  for (int si = 0; si < (int)P.nodes.size(); ++si) {
    const NDNode& S = P.nodes[si];
    const int gmax = S.leaf() ? S.level : std::max(S.level, P.depth - 1);
    std::vector<std::vector<int>> cur{*sep_of[si]};
    // descendants of S
    std::vector<int> sub, st{si};
    while (!st.empty()) {
      const int n = st.back();
      st.pop_back();
      sub.push_back(n);
      for (int c = 0; c < 2; ++c)
        if (P.nodes[n].child[c] >= 0) st.push_back(P.nodes[n].child[c]);
    }
    for (int g = S.level;; ++g) {
      for (auto& pc : cur) pieces.push_back({S.rank, pc.front(), si, g, pc});
      if (g == gmax) break;
      for (int t : sub)
        if (P.nodes[t].level == g + 1 && !P.nodes[t].leaf())
          for (int c : *sep_of[t]) tcol[c] = 1;
      std::vector<std::vector<int>> nxt;
      for (const auto& pc : cur) {
        std::vector<int> a, b;
        for (int v : pc) {
          bool cut = false;
          for (int64_t k = G.ptr[v]; k < G.ptr[v + 1] && !cut; ++k) cut = tcol[G.idx[k]] != 0;
          (cut ? a : b).push_back(v);
        }
        if (!a.empty()) components(G, a, in, seen, nxt);
        if (!b.empty()) components(G, b, in, seen, nxt);
      }
      for (int t : sub)
        if (P.nodes[t].level == g + 1 && !P.nodes[t].leaf())
          for (int c : *sep_of[t]) tcol[c] = 0;
      std::sort(nxt.begin(), nxt.end(), [](const std::vector<int>& x, const std::vector<int>& y) {
        return x.front() < y.front();
      });
      cur.swap(nxt);
    }
  }
  std::sort(pieces.begin(), pieces.end(), [](const Piece& a, const Piece& b) {
    if (a.k0 != b.k0) return a.k0 < b.k0;
    if (a.k1 != b.k1) return a.k1 < b.k1;
    return a.gran < b.gran;
  });
  P.clusters.assign(pieces.size(), Cluster());
  for (auto& S : P.nodes) {
    const int gmax = S.leaf() ? S.level : std::max(S.level, P.depth - 1);
    S.pieces.assign(gmax - S.level + 1, {});
  }
  std::vector<int> owner_at(N, -1);  // piece of the previous granularity holding each column
  for (size_t i = 0; i < pieces.size(); ++i) {
    Cluster& c = P.clusters[i];
    c.key0 = pieces[i].k0;
    c.key1 = pieces[i].k1;
    c.sep = pieces[i].sep;
    c.gran = pieces[i].gran;
    for (int a = 0; a < 3; ++a) c.lo[a] = c.hi[a] = 0;
    P.nodes[c.sep].pieces[c.gran - P.nodes[c.sep].level].push_back((int)i);
  }
  // hierarchy by column membership; the finest pieces carry the columns
  P.col_cluster.assign(N, -1);
  P.finest.clear();
  for (int si = 0; si < (int)P.nodes.size(); ++si) {
    NDNode& S = P.nodes[si];
    for (size_t gi = 0; gi < S.pieces.size(); ++gi) {
      if (gi > 0)
        for (int ci : S.pieces[gi]) {
          const std::vector<int>& cols = pieces[ci].cols;
          const int par = owner_at[cols.front()];
          for (int v : cols)
            if (owner_at[v] != par) throw Error(SPAQR_EARG, "interface hierarchy does not nest");
          P.clusters[ci].parent = par;
          P.clusters[par].children.push_back(ci);
        }
      for (int ci : S.pieces[gi])
        for (int v : pieces[ci].cols) owner_at[v] = ci;
    }
    for (auto& lst : S.pieces)
      for (int ci : lst) std::sort(P.clusters[ci].children.begin(), P.clusters[ci].children.end());
  }
  for (size_t i = 0; i < P.clusters.size(); ++i) {
    Cluster& c = P.clusters[i];
    const NDNode& S = P.nodes[c.sep];
    const int gmax = S.leaf() ? S.level : std::max(S.level, P.depth - 1);
    if (c.gran != gmax) continue;
    c.finest_index = (int)P.finest.size();
    P.finest.push_back((int)i);
    c.cells = pieces[i].cols;
    for (int j : c.cells) {
      if (P.col_cluster[j] >= 0) throw Error(SPAQR_EARG, "column in two clusters");
      P.col_cluster[j] = (int)i;
    }
  }
  for (int j = 0; j < N; ++j)
    if (P.col_cluster[j] < 0) throw Error(SPAQR_EARG, "column in no cluster");
}

std::vector<int64_t> max_product_matching(const Plan& P) {
  const int64_t M = P.M, N = P.N;
  // columns' rows and costs
  std::vector<int64_t> cptr(N + 1, 0);
  for (int64_t e = 0; e < P.nnz; ++e) cptr[P.col_idx[e] + 1]++;
  for (int64_t j = 0; j < N; ++j) cptr[j + 1] += cptr[j];
  std::vector<int64_t> crow(P.nnz);
  std::vector<double> cval(P.nnz);
  std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
  for (int64_t r = 0; r < M; ++r)
    for (int64_t e = P.row_ptr[r]; e < P.row_ptr[r + 1]; ++e) {
      const int64_t d = fill[P.col_idx[e]]++;
      crow[d] = r;
      if (P.vals[e] == 0.0) throw Error(SPAQR_EARG, "explicit zero entry in A");
      cval[d] = std::log(std::fabs(P.vals[e]));
    }
  std::vector<double> cost(P.nnz), u(N, 0.0), v(M, 0.0);
  for (int64_t j = 0; j < N; ++j) {
    double mx = -std::numeric_limits<double>::infinity();
    for (int64_t k = cptr[j]; k < cptr[j + 1]; ++k) mx = std::max(mx, cval[k]);
    double mn = std::numeric_limits<double>::infinity();
    for (int64_t k = cptr[j]; k < cptr[j + 1]; ++k) {
      cost[k] = mx - cval[k];
      mn = std::min(mn, cost[k]);
    }
    u[j] = mn;
  }
  std::vector<int64_t> row_match(M, -1), col_match(N, -1);
  const double INF = std::numeric_limits<double>::infinity();
  std::vector<double> dist(M, INF);
  std::vector<int64_t> pred(M, -1);
  std::vector<char> done(M, 0);
  std::vector<int64_t> touched, final_rows;
  typedef std::pair<double, int64_t> QE;
  for (int64_t j = 0; j < N; ++j) {
    std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
    touched.clear();
    final_rows.clear();
    auto relax = [&](int64_t c, double base) {
      for (int64_t k = cptr[c]; k < cptr[c + 1]; ++k) {
        const int64_t r = crow[k];
        if (done[r]) continue;
        const double nd = base + (cost[k] - u[c] - v[r]);
        if (nd < dist[r]) {
          if (dist[r] == INF) touched.push_back(r);
          dist[r] = nd;
          pred[r] = c;
          pq.push({nd, r});
        }
      }
    };
    relax(j, 0.0);
    int64_t sink = -1;
    double dmin = 0.0;
    while (!pq.empty()) {
      const QE top = pq.top();
      pq.pop();
      const int64_t r = top.second;
      if (done[r] || top.first > dist[r]) continue;
      done[r] = 1;
      final_rows.push_back(r);
      if (row_match[r] < 0) {
        sink = r;
        dmin = dist[r];
        break;
      }
      relax(row_match[r], dist[r]);
    }
    if (sink < 0) throw Error(SPAQR_EARG, "no row matching covers every column (structurally rank deficient)");
    // potentials: nodes settled closer than the sink move by their gap
    u[j] += dmin;
    for (int64_t r : final_rows) {
      if (r == sink) continue;
      const double gap = dmin - dist[r];
      v[r] -= gap;
      u[row_match[r]] += gap;
    }
    // augment along the alternating path
    int64_t r = sink;
    for (;;) {
      const int64_t c = pred[r];
      const int64_t prev = col_match[c];
      col_match[c] = r;
      row_match[r] = c;
      if (c == j) break;
      r = prev;
    }
    for (int64_t t : touched) dist[t] = INF, pred[t] = -1, done[t] = 0;
  }
  return col_match;
}

}  // namespace spaqr
