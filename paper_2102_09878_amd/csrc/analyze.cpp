// Host analysis of spaQR (Section 2.2 and 2.7 of Gnanasekaran & Darve):
// column scaling, geometric nested dissection on the cell grid, interfaces
// of every separator at every granularity and their hierarchy, row matching
// and max-norm assignment of the remaining rows, and the symbolic layout of
// the initial row groups.  Pure host code: no GPU is touched here.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

#include "spaqr_impl.h"

namespace spaqr {

namespace {

struct TmpNode {
  int level;
  int64_t path;
  int lo[3], hi[3];
  int axis = -1, t = -1;
  int child[2] = {-1, -1};
  int parent = -1;
};

int64_t cell_index(const int* c, const int* grid) {
  return c[0] + (int64_t)grid[0] * (c[1] + (int64_t)grid[1] * c[2]);
}

// Split rule: longest axis (ties x, y, z), `w` planes starting at lo + (len - w) / 2.
void build_tree(Plan& P) {
  std::vector<TmpNode> tmp;
  struct Item {
    int lo[3], hi[3], level;
    int64_t path;
    int parent, side;
  };
  std::vector<Item> stack;
  Item root;
  for (int a = 0; a < 3; ++a) root.lo[a] = 0, root.hi[a] = P.grid[a];
  root.level = 1;
  root.path = 0;
  root.parent = -1;
  root.side = 0;
  stack.push_back(root);
  while (!stack.empty()) {
    Item it = stack.back();
    stack.pop_back();
    TmpNode n;
    n.level = it.level;
    n.path = it.path;
    for (int a = 0; a < 3; ++a) n.lo[a] = it.lo[a], n.hi[a] = it.hi[a];
    n.parent = it.parent;
    int id = (int)tmp.size();
    if (it.parent >= 0) tmp[it.parent].child[it.side] = id;
    if (it.level < P.depth) {
      int axis = 0;
      for (int a = 1; a < 3; ++a)
        if (it.hi[a] - it.lo[a] > it.hi[axis] - it.lo[axis]) axis = a;
      int len = it.hi[axis] - it.lo[axis];
      if (len < P.w + 2)
        throw Error(SPAQR_EARG, "grid too small for the requested nested-dissection depth");
      n.axis = axis;
      n.t = it.lo[axis] + (len - P.w) / 2;
      tmp.push_back(n);
      Item hiC = it, loC = it;
      loC.hi[axis] = n.t;
      hiC.lo[axis] = n.t + P.w;
      loC.level = hiC.level = it.level + 1;
      loC.path = 2 * it.path;
      hiC.path = 2 * it.path + 1;
      loC.parent = hiC.parent = id;
      loC.side = 0;
      hiC.side = 1;
      stack.push_back(hiC);
      stack.push_back(loC);
    } else {
      tmp.push_back(n);
    }
  }
  std::vector<int> order(tmp.size());
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (tmp[a].level != tmp[b].level) return tmp[a].level > tmp[b].level;
    return tmp[a].path < tmp[b].path;
  });
  std::vector<int> rank_of(tmp.size());
  for (size_t r = 0; r < order.size(); ++r) rank_of[order[r]] = (int)r;
  P.nodes.assign(tmp.size(), NDNode());
  for (size_t i = 0; i < tmp.size(); ++i) {
    NDNode& d = P.nodes[rank_of[i]];
    const TmpNode& s = tmp[i];
    d.level = s.level;
    d.path = s.path;
    for (int a = 0; a < 3; ++a) d.lo[a] = s.lo[a], d.hi[a] = s.hi[a];
    d.axis = s.axis;
    d.t = s.t;
    d.parent = s.parent >= 0 ? rank_of[s.parent] : -1;
    for (int c = 0; c < 2; ++c) d.child[c] = s.child[c] >= 0 ? rank_of[s.child[c]] : -1;
    d.rank = rank_of[i];
  }
}

void sep_box(const Plan& P, const NDNode& S, int* lo, int* hi) {
  for (int a = 0; a < 3; ++a) lo[a] = S.lo[a], hi[a] = S.hi[a];
  if (!S.leaf()) {
    lo[S.axis] = S.t;
    hi[S.axis] = S.t + P.w;
  }
}

void subtree(const Plan& P, int root, std::vector<int>& out) {
  std::vector<int> st{root};
  while (!st.empty()) {
    int n = st.back();
    st.pop_back();
    out.push_back(n);
    for (int c = 0; c < 2; ++c)
      if (P.nodes[n].child[c] >= 0) st.push_back(P.nodes[n].child[c]);
  }
}

int finest_gran(const Plan& P, const NDNode& S) {
  return S.leaf() ? S.level : std::max(S.level, P.depth - 1);
}

// Interfaces of S at granularity g: per face axis, intervals refined level by
// level by the cut planes of touching descendant separators on that axis.
std::vector<std::pair<std::array<int, 3>, std::array<int, 3>>> piece_boxes(const Plan& P, int sidx,
                                                                           int g) {
  const NDNode& S = P.nodes[sidx];
  int lo[3], hi[3];
  sep_box(P, S, lo, hi);
  std::vector<std::vector<std::pair<int, int>>> iv(3);
  std::vector<int> sub;
  if (!S.leaf()) subtree(P, sidx, sub);
  for (int b = 0; b < 3; ++b) {
    iv[b].push_back({lo[b], hi[b]});
    if (S.leaf() || b == S.axis) continue;
    for (int lam = S.level + 1; lam <= g; ++lam) {
      std::vector<char> cut(P.grid[b] + 1, 0);
      for (int ti : sub) {
        const NDNode& T = P.nodes[ti];
        if (ti == sidx || T.level != lam || T.leaf() || T.axis != b) continue;
        if (T.hi[S.axis] == S.t || T.lo[S.axis] == S.t + P.w)
          for (int c = T.t; c < T.t + P.w; ++c) cut[c] = 1;
      }
      std::vector<std::pair<int, int>> nx;
      for (auto [a0, a1] : iv[b]) {
        int start = a0;
        for (int c = a0 + 1; c < a1; ++c)
          if (cut[c] != cut[c - 1]) {
            nx.push_back({start, c});
            start = c;
          }
        nx.push_back({start, a1});
      }
      iv[b].swap(nx);
    }
  }
  std::vector<std::pair<std::array<int, 3>, std::array<int, 3>>> out;
  for (auto ix : iv[0])
    for (auto iy : iv[1])
      for (auto iz : iv[2])
        out.push_back({{ix.first, iy.first, iz.first}, {ix.second, iy.second, iz.second}});
  return out;
}

bool ancestor_or_self(const NDNode& a, const NDNode& b) {
  if (b.level < a.level) return false;
  return (b.path >> (b.level - a.level)) == a.path;
}

// geometric tree, interfaces, hierarchy and finest clusters (below)
void build_geometric(Plan& P);

}  // namespace

void rescale_values(Plan& P, const double* vals) {
  P.vals.assign(vals, vals + P.nnz);
  P.D.assign(P.N, 0.0);
  for (int64_t e = 0; e < P.nnz; ++e) P.D[P.col_idx[e]] += P.vals[e] * P.vals[e];
  for (int64_t j = 0; j < P.N; ++j) {
    if (!(P.D[j] > 0.0)) throw Error(SPAQR_EARG, "column " + std::to_string(j) + " is empty");
    P.D[j] = std::sqrt(P.D[j]);
  }
  P.ahat.resize(P.nnz);
  for (int64_t e = 0; e < P.nnz; ++e) P.ahat[e] = P.vals[e] / P.D[P.col_idx[e]];
}

void analyze_plan(Plan& P, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                  int64_t M, int64_t N, const spaqr_options& opt) {
  if (!row_ptr || !col_idx || !vals) throw Error(SPAQR_EARG, "null CSR pointer");
  if (N < 1 || M < N) throw Error(SPAQR_EARG, "need M >= N >= 1");
  P.M = M;
  P.N = N;
  // with a cell grid the partition is geometric; without one (grid[0] <= 0)
  // it is the graph nested dissection of graph_nd.cpp
  const bool geometric = opt.grid[0] > 0;
  for (int a = 0; a < 3; ++a) P.grid[a] = opt.grid[a] > 0 ? opt.grid[a] : (geometric ? 1 : 0);
  if (geometric && opt.grid[1] <= 0) throw Error(SPAQR_EARG, "grid[1] must be positive with grid[0]");
  if (geometric && (int64_t)P.grid[0] * P.grid[1] * P.grid[2] != N)
    throw Error(SPAQR_EARG, "grid size does not match N");
  if (!geometric && N >= ((int64_t)1 << 31)) throw Error(SPAQR_EARG, "N too large");
  P.w = opt.sep_width > 0 ? opt.sep_width : 2;
  P.depth = opt.nd_depth > 0 ? opt.nd_depth
                             : std::max(2, (int)std::ceil(std::log2((double)N / 64.0)));
  P.skip = opt.sparsify_skip >= 0 ? opt.sparsify_skip : (P.depth <= 4 ? 1 : 2);

  // CSR validation
  if (row_ptr[0] != 0) throw Error(SPAQR_EARG, "row_ptr[0] must be 0");
  for (int64_t r = 0; r < M; ++r) {
    if (row_ptr[r + 1] < row_ptr[r]) throw Error(SPAQR_EARG, "row_ptr not monotone");
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      if (col_idx[e] < 0 || col_idx[e] >= N) throw Error(SPAQR_EARG, "column index out of range");
      if (e > row_ptr[r] && col_idx[e] <= col_idx[e - 1])
        throw Error(SPAQR_EARG, "columns not sorted and unique within a row");
    }
  }
  P.nnz = row_ptr[M];
  P.row_ptr.assign(row_ptr, row_ptr + M + 1);
  P.col_idx.assign(col_idx, col_idx + P.nnz);
  rescale_values(P, vals);

  std::vector<int64_t> match;
  if (geometric) {
    build_geometric(P);
    match.resize(N);
    std::iota(match.begin(), match.end(), 0);  // column j <-> its Laplacian row j
  } else {
    graph_partition(P);
    match = max_product_matching(P);
  }
  finish_plan(P, match);
}

namespace {

void build_geometric(Plan& P) {
  const int64_t N = P.N;
  build_tree(P);

  // clusters of every separator at every granularity
  struct Tmp {
    int64_t k0, k1;
    int sep, gran;
    std::array<int, 3> lo, hi;
  };
  std::vector<Tmp> tmp;
  for (size_t si = 0; si < P.nodes.size(); ++si) {
    const NDNode& S = P.nodes[si];
    for (int g = S.level; g <= finest_gran(P, S); ++g)
      for (auto& bx : piece_boxes(P, (int)si, g))
        tmp.push_back({S.rank, cell_index(bx.first.data(), P.grid), (int)si, g, bx.first, bx.second});
  }
  std::sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) {
    if (a.k0 != b.k0) return a.k0 < b.k0;
    if (a.k1 != b.k1) return a.k1 < b.k1;
    return a.gran < b.gran;
  });
  P.clusters.assign(tmp.size(), Cluster());
  for (auto& S : P.nodes) S.pieces.assign(finest_gran(P, S) - S.level + 1, {});
  for (size_t i = 0; i < tmp.size(); ++i) {
    Cluster& c = P.clusters[i];
    c.key0 = tmp[i].k0;
    c.key1 = tmp[i].k1;
    c.sep = tmp[i].sep;
    c.gran = tmp[i].gran;
    for (int a = 0; a < 3; ++a) c.lo[a] = tmp[i].lo[a], c.hi[a] = tmp[i].hi[a];
    P.nodes[c.sep].pieces[c.gran - P.nodes[c.sep].level].push_back((int)i);
  }
  // hierarchy: parent = the coarser piece containing the box
  for (auto& S : P.nodes) {
    for (size_t gi = 0; gi + 1 < S.pieces.size(); ++gi) {
      for (int ci : S.pieces[gi + 1]) {
        Cluster& c = P.clusters[ci];
        int found = -1;
        for (int pi : S.pieces[gi]) {
          const Cluster& p = P.clusters[pi];
          bool in = true;
          for (int a = 0; a < 3; ++a) in = in && p.lo[a] <= c.lo[a] && c.hi[a] <= p.hi[a];
          if (in) {
            if (found >= 0) throw Error(SPAQR_EARG, "interface hierarchy does not nest");
            found = pi;
          }
        }
        if (found < 0) throw Error(SPAQR_EARG, "interface hierarchy does not nest");
        c.parent = found;
        P.clusters[found].children.push_back(ci);
      }
    }
    for (auto& lst : S.pieces)
      for (int ci : lst) std::sort(P.clusters[ci].children.begin(), P.clusters[ci].children.end());
  }
  // finest clusters and their cells
  P.col_cluster.assign(N, -1);
  P.finest.clear();
  for (size_t i = 0; i < P.clusters.size(); ++i) {
    Cluster& c = P.clusters[i];
    const NDNode& S = P.nodes[c.sep];
    if (c.gran != finest_gran(P, S)) continue;
    c.finest_index = (int)P.finest.size();
    P.finest.push_back((int)i);
    for (int z = c.lo[2]; z < c.hi[2]; ++z)
      for (int y = c.lo[1]; y < c.hi[1]; ++y)
        for (int x = c.lo[0]; x < c.hi[0]; ++x) {
          int cc[3] = {x, y, z};
          int64_t j = cell_index(cc, P.grid);
          if (P.col_cluster[j] >= 0) throw Error(SPAQR_EARG, "cell in two clusters");
          P.col_cluster[j] = (int)i;
          c.cells.push_back((int)j);
        }
  }
  for (int64_t j = 0; j < N; ++j)
    if (P.col_cluster[j] < 0) throw Error(SPAQR_EARG, "cell in no cluster");
}

}  // namespace

void finish_plan(Plan& P, const std::vector<int64_t>& match) {
  const int64_t M = P.M, N = P.N;
  const int64_t* row_ptr = P.row_ptr.data();
  const int32_t* col_idx = P.col_idx.data();
  // rows must not couple two sibling subtrees
  for (int64_t r = 0; r < M; ++r) {
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
      for (int64_t f = e + 1; f < row_ptr[r + 1]; ++f) {
        const NDNode& a = P.nodes[P.clusters[P.col_cluster[col_idx[e]]].sep];
        const NDNode& b = P.nodes[P.clusters[P.col_cluster[col_idx[f]]].sep];
        if (!ancestor_or_self(a, b) && !ancestor_or_self(b, a))
          throw Error(SPAQR_EARG, "row " + std::to_string(r) + " couples two sibling subtrees");
      }
  }

  // row ownership: the row matched to column j goes to j's cluster; other
  // rows to the finest cluster with the largest sum of squared scaled
  // entries (lowest id on ties)
  P.row_owner.assign(M, -1);
  for (int64_t j = 0; j < N; ++j) P.row_owner[match[j]] = P.col_cluster[j];
  for (int64_t r = 0; r < M; ++r) {
    if (P.row_owner[r] >= 0) continue;
    std::vector<std::pair<int, double>> acc;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      int c = P.col_cluster[col_idx[e]];
      double v = P.ahat[e] * P.ahat[e];
      bool hit = false;
      for (auto& kv : acc)
        if (kv.first == c) kv.second += v, hit = true;
      if (!hit) acc.push_back({c, v});
    }
    if (acc.empty()) throw Error(SPAQR_EARG, "empty row " + std::to_string(r));
    int best = -1;
    double bv = -1.0;
    for (auto& kv : acc)
      if (kv.second > bv || (kv.second == bv && kv.first < best)) best = kv.first, bv = kv.second;
    P.row_owner[r] = best;
  }

  // initial groups: rows of one owner touching the same set of clusters,
  // ordered by first row; rows ascending
  std::map<std::pair<int, std::vector<int>>, int> gid;
  P.init_groups.clear();
  std::vector<int> row_group(M), row_pos(M);
  for (int64_t r = 0; r < M; ++r) {
    std::vector<int> sig;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) sig.push_back(P.col_cluster[col_idx[e]]);
    std::sort(sig.begin(), sig.end());
    sig.erase(std::unique(sig.begin(), sig.end()), sig.end());
    auto key = std::make_pair(P.row_owner[r], sig);
    auto it = gid.find(key);
    int g;
    if (it == gid.end()) {
      g = (int)P.init_groups.size();
      gid.emplace(key, g);
      InitGroup ig;
      ig.owner = P.row_owner[r];
      ig.clus = sig;
      P.init_groups.push_back(ig);
    } else {
      g = it->second;
    }
    row_group[r] = g;
    row_pos[r] = (int)P.init_groups[g].rows.size();
    P.init_groups[g].rows.push_back((int)r);
  }
  int64_t off = 0;
  for (auto& g : P.init_groups) {
    g.width = 0;
    for (int c : g.clus) g.width += (int)P.clusters[c].cells.size();
    g.ld = ((int64_t)g.rows.size() + 3) / 4 * 4;
    g.offset = off;
    off += g.ld * g.width;
    off = (off + 63) / 64 * 64;
  }
  P.init_elems = off;
  // destination of every CSR entry inside its group
  P.init_dst.assign(P.nnz, 0);
  for (int64_t r = 0; r < M; ++r) {
    const InitGroup& g = P.init_groups[row_group[r]];
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      int j = col_idx[e];
      int cl = P.col_cluster[j];
      int col = 0;
      for (int c : g.clus) {
        if (c == cl) break;
        col += (int)P.clusters[c].cells.size();
      }
      const auto& cells = P.clusters[cl].cells;
      col += (int)(std::lower_bound(cells.begin(), cells.end(), j) - cells.begin());
      P.init_dst[e] = g.offset + row_pos[r] + (int64_t)col * g.ld;
    }
  }
  P.count = 1;
  P.seg_col = {0, N};
  P.seg_row = {0, M};
  P.seg_depth = {P.depth};
  // A^T pattern
  P.at_ptr.assign(N + 1, 0);
  for (int64_t e = 0; e < P.nnz; ++e) P.at_ptr[col_idx[e] + 1]++;
  for (int64_t j = 0; j < N; ++j) P.at_ptr[j + 1] += P.at_ptr[j];
  P.at_idx.resize(P.nnz);
  P.at_src.resize(P.nnz);
  std::vector<int64_t> fill(P.at_ptr.begin(), P.at_ptr.end() - 1);
  for (int64_t r = 0; r < M; ++r)
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      int64_t d = fill[col_idx[e]]++;
      P.at_idx[d] = (int32_t)r;
      P.at_src[d] = e;
    }
}

void union_plans(Plan& U, std::vector<Plan>& parts) {
  if (parts.empty()) throw Error(SPAQR_EARG, "empty batch");
  U = Plan();
  int dmax = 0;
  for (const Plan& p : parts) {
    dmax = std::max(dmax, p.depth);
    if (p.skip != parts[0].skip) throw Error(SPAQR_EARG, "batch members must share sparsify_skip");
    if (p.w != parts[0].w) throw Error(SPAQR_EARG, "batch members must share sep_width");
  }
  U.depth = dmax;
  U.skip = parts[0].skip;
  U.w = parts[0].w;
  U.count = (int)parts.size();
  U.seg_col = {0};
  U.seg_row = {0};
  int64_t nnz = 0, elems = 0;
  for (const Plan& p : parts) {
    const int shift = dmax - p.depth;
    const int nb = (int)U.nodes.size(), cb = (int)U.clusters.size(), fb = (int)U.finest.size();
    const int64_t colb = U.N, rowb = U.M, nzb = nnz, eb = elems;
    for (NDNode n : p.nodes) {
      n.level += shift;
      n.rank += nb;
      for (int& c : n.child)
        if (c >= 0) c += nb;
      if (n.parent >= 0) n.parent += nb;
      for (auto& lst : n.pieces)
        for (int& c : lst) c += cb;
      U.nodes.push_back(std::move(n));
    }
    for (Cluster c : p.clusters) {
      c.sep += nb;
      c.gran += shift;
      if (c.parent >= 0) c.parent += cb;
      for (int& k : c.children) k += cb;
      for (int& j : c.cells) j += (int)colb;
      if (c.finest_index >= 0) c.finest_index += fb;
      U.clusters.push_back(std::move(c));
    }
    for (int f : p.finest) U.finest.push_back(f + cb);
    for (int c : p.col_cluster) U.col_cluster.push_back(c + cb);
    for (int c : p.row_owner) U.row_owner.push_back(c + cb);
    for (InitGroup g : p.init_groups) {
      g.owner += cb;
      for (int& r : g.rows) r += (int)rowb;
      for (int& c : g.clus) c += cb;
      g.offset += eb;
      U.init_groups.push_back(std::move(g));
    }
    for (int64_t d : p.init_dst) U.init_dst.push_back(d + eb);
    for (int64_t r = 0; r < p.M; ++r) U.row_ptr.push_back(p.row_ptr[r] + nzb);
    for (int32_t c : p.col_idx) U.col_idx.push_back(c + (int32_t)colb);
    U.vals.insert(U.vals.end(), p.vals.begin(), p.vals.end());
    U.ahat.insert(U.ahat.end(), p.ahat.begin(), p.ahat.end());
    U.D.insert(U.D.end(), p.D.begin(), p.D.end());
    for (int64_t j = 0; j < p.N; ++j) U.at_ptr.push_back(p.at_ptr[j] + nzb);
    for (int32_t r : p.at_idx) U.at_idx.push_back(r + (int32_t)rowb);
    for (int64_t e : p.at_src) U.at_src.push_back(e + nzb);
    U.M += p.M;
    U.N += p.N;
    nnz += p.nnz;
    elems += (p.init_elems + 63) / 64 * 64;
    U.seg_col.push_back(U.N);
    U.seg_row.push_back(U.M);
    U.seg_depth.push_back(p.depth);
  }
  if (U.N >= (int64_t)1 << 31 || U.M >= (int64_t)1 << 31) throw Error(SPAQR_EARG, "batch too large");
  U.row_ptr.push_back(nnz);
  U.at_ptr.push_back(nnz);
  U.nnz = nnz;
  U.init_elems = elems;
  U.grid[0] = U.grid[1] = U.grid[2] = 0;  // no single grid
}

}  // namespace spaqr
