// Level-by-level spaQR factorization on one GPU (Algorithm 1 of
// Gnanasekaran & Darve, Sections 2.3-2.7).
//
// Device data, host metadata: every row group (a dense block of rows owned
// by one cluster, stored over an explicit list of column slots) lives in
// device memory; the host keeps the block structure (which clusters each
// group touches, live column slots of each cluster) and turns each phase
// into a few batched launches over descriptor arrays: gather fronts -> QR
// -> write back.  The host reads back only what decides structure: owners
// of reassigned rows and the ranks chosen by the rank-revealing QRs.
//
// Scheduling readings (the paper leaves the order open):
//  * the clusters of one level are eliminated in rounds; a round takes, in
//    id order, every pending cluster sharing no front row and no front
//    column with one already taken; one round = one batched launch chain;
//  * step 2 runs in rounds the same way, p ~ q when q is a column cluster
//    of p's scaled rows or p one of q's;
//  * scaling applies every left transform U_pp^T, then every right R_pp^-1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <unordered_map>

#include "handle.h"

namespace spaqr {

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------
static constexpr size_t kChunk = size_t(256) << 20;

Arena::~Arena() { release(); }
void* Arena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  while (cur_ < chunks_.size() && chunks_[cur_].off + bytes > chunks_[cur_].size) ++cur_;
  if (cur_ == chunks_.size()) {
    Chunk c{nullptr, std::max(kChunk, bytes), 0};
    if (hipMalloc(&c.ptr, c.size) != hipSuccess) throw Error(SPAQR_ENOMEM, "device allocation failed");
    chunks_.push_back(c);
  }
  Chunk& c = chunks_[cur_];
  void* p = c.ptr + c.off;
  c.off += bytes;
  used_total_ += bytes;
  return p;
}
void Arena::reset() {
  for (auto& c : chunks_) c.off = 0;
  cur_ = 0;
  used_total_ = 0;
}
void Arena::release() {
  for (auto& c : chunks_) (void)hipFree(c.ptr);
  chunks_.clear();
  cur_ = 0;
  used_total_ = 0;
}
size_t Arena::capacity() const {
  size_t s = 0;
  for (auto& c : chunks_) s += c.size;
  return s;
}

Staging::~Staging() { release(); }
void* Staging::alloc(size_t bytes) {
  bytes = (bytes + 63) & ~size_t(63);
  if (bytes == 0) bytes = 64;
  while (cur_ < chunks_.size() && chunks_[cur_].off + bytes > chunks_[cur_].size) ++cur_;
  if (cur_ == chunks_.size()) {
    Chunk c{nullptr, std::max(size_t(64) << 20, bytes), 0};
    if (hipHostMalloc((void**)&c.ptr, c.size, hipHostMallocDefault) != hipSuccess)
      throw Error(SPAQR_ENOMEM, "pinned host allocation failed");
    chunks_.push_back(c);
  }
  Chunk& c = chunks_[cur_];
  void* p = c.ptr + c.off;
  c.off += bytes;
  return p;
}
void Staging::reset() {
  for (auto& c : chunks_) c.off = 0;
  cur_ = 0;
}
void Staging::release() {
  for (auto& c : chunks_) (void)hipHostFree(c.ptr);
  chunks_.clear();
  cur_ = 0;
}

Handle::~Handle() {
  try {
    release_device();
  } catch (...) {
  }
}

void Handle::drop_cg_graph() {
  if (cg_exec) (void)hipGraphExecDestroy(cg_exec);
  if (cg_graph) (void)hipGraphDestroy(cg_graph);
  cg_exec = nullptr;
  cg_graph = nullptr;
  cg_base = nullptr;
}

void Handle::release_device() {
  if (!dev_ready) return;
  (void)hipStreamSynchronize(stream);
  drop_cg_graph();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  cap_stream = nullptr;
  for (void* p : {(void*)d_ahat, (void*)d_rp, (void*)d_ci, (void*)d_ahatT, (void*)d_atp, (void*)d_ati,
                  (void*)d_init_dst, (void*)d_D, (void*)d_cg, (void*)d_vals, (void*)d_atsrc, (void*)d_flag,
                  (void*)d_segc, (void*)d_segr, (void*)d_act, (void*)d_pqr_err})
    if (p) (void)hipFree(p);
  d_pqr_err = nullptr;
  if (h_sc) (void)hipHostFree(h_sc);
  if (h_act) (void)hipHostFree(h_act);
  if (h_pqr_report) (void)hipHostFree(h_pqr_report);
  h_pqr_report = d_pqr_report = nullptr;
  d_segc = d_segr = nullptr;
  d_act = nullptr;
  h_act = nullptr;
  cg_elems = 0;
  d_ahat = d_ahatT = d_D = d_cg = d_vals = nullptr;
  d_atsrc = nullptr;
  d_flag = nullptr;
  d_rp = d_atp = nullptr;
  d_ci = d_ati = nullptr;
  d_init_dst = nullptr;
  h_sc = nullptr;
  arena.release();
  stage.release();
  dev_ready = false;
}

template <class V>
static V* dcopy(const std::vector<V>& h, size_t& bytes) {
  V* d = nullptr;
  const size_t b = std::max<size_t>(1, h.size()) * sizeof(V);
  if (hipMalloc(&d, b) != hipSuccess) throw Error(SPAQR_ENOMEM, "device allocation failed");
  if (!h.empty()) SPAQR_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  bytes += b;
  return d;
}

void Handle::ensure_device() {
  if (dev_ready) return;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) throw Error(SPAQR_EHIP, "no HIP device");
  SPAQR_HIP(hipSetDevice(opt.device));
  stream = static_cast<hipStream_t>(opt.stream);
  plan_bytes = 0;
  d_rp = dcopy(P.row_ptr, plan_bytes);
  d_ci = dcopy(P.col_idx, plan_bytes);
  d_vals = dcopy(P.vals, plan_bytes);
  d_atp = dcopy(P.at_ptr, plan_bytes);
  d_ati = dcopy(P.at_idx, plan_bytes);
  d_atsrc = dcopy(P.at_src, plan_bytes);
  d_init_dst = dcopy(P.init_dst, plan_bytes);
  d_ahat = dcopy(std::vector<double>(P.nnz), plan_bytes);
  d_ahatT = dcopy(std::vector<double>(P.nnz), plan_bytes);
  d_D = dcopy(std::vector<double>(P.N), plan_bytes);
  d_flag = dcopy(std::vector<int>(1), plan_bytes);
  d_segc = dcopy(P.seg_col, plan_bytes);
  d_segr = dcopy(P.seg_row, plan_bytes);
  d_act = dcopy(std::vector<int>(P.count, 1), plan_bytes);
  d_pqr_err = dcopy(std::vector<int>(1), plan_bytes);
  SPAQR_HIP(hipHostMalloc((void**)&h_sc, (P.count * 8 + 64) * sizeof(double), hipHostMallocDefault));
  SPAQR_HIP(hipHostMalloc((void**)&h_act, P.count * sizeof(int), hipHostMallocDefault));
  SPAQR_HIP(hipHostMalloc((void**)&h_pqr_report, 64, hipHostMallocCoherent | hipHostMallocMapped));
  *h_pqr_report = 0;
  SPAQR_HIP(hipHostGetDevicePointer((void**)&d_pqr_report, h_pqr_report, 0));
  dev_ready = true;
  scale_values(*this);
}

// ---------------------------------------------------------------------------
// factorization
// ---------------------------------------------------------------------------

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

double qr_flops(double m, double n) {
  return m >= n ? 2.0 * m * n * n - 2.0 * n * n * n / 3.0 : 2.0 * n * m * m - 2.0 * m * m * m / 3.0;
}

enum Phase { PH_ELIM = 0, PH_REASSIGN = 1, PH_SCALE = 2, PH_SPARSIFY = 3, PH_MERGE = 4 };

// Every rank-revealing QR stops at the numerical rank: a pivot with
// |R_ii| <= kNoiseRank * u * ||C||_F is rounding error, and reflectors built
// from it (and rows or columns kept because of it) would differ from run to
// run and from any other implementation.
constexpr double kNoiseRank = 1000.0;
// batches of at least this many matrices read a matrix's state before its
// columns in a pivot step (see k_pqr_step)
constexpr int kCheckFirstMats = 2;
template <typename T>
constexpr double unit_roundoff() {
  return sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
}

template <typename T>
class Factorizer {
 public:
  Factorizer(Handle& h, double eps, const int* forced, int nforced)
      : H(h), P(h.P), raw_st_(h.stream), eps_(eps), forced_(forced), nforced_(nforced) {}

  void run();

 private:
  typedef std::shared_ptr<const SlotList> Slots;
  // the list `cols` made of the slot lists of `head` (if >= 0) then of the
  // clusters `cl`, in that order (the blocks are cut by their sizes)
  Slots make_slots(const std::vector<int>& cols, size_t from, int head, const std::vector<int>& cl) {
    auto L = std::make_shared<SlotList>();
    L->v.assign(cols.begin() + from, cols.end());
    int at = 0;
    auto block = [&](int c, int len) {
      L->blk.push_back({c, at, at + len});
      at += len;
    };
    if (head >= 0) block(head, (int)C[head].slots.size());
    for (int q : cl) block(q, (int)C[q].slots.size());
    if (at != (int)L->v.size()) throw Error(SPAQR_EARG, "internal: slot list blocks do not cover the list");
    return L;
  }
  // c is p or one of the clusters merged into p
  bool within(int c, int p) const {
    for (; c >= 0; c = P.clusters[c].parent)
      if (c == p) return true;
    return false;
  }
  struct RG {
    int owner = -1;
    T* data = nullptr;
    int64_t ld = 0;
    int nrows = 0;
    // column slots of the data, shared by the groups made from one front
    // (so a map into them is found once per list)
    Slots sl;
    const std::vector<int>& slots() const {
      static const std::vector<int> none;
      return sl ? sl->v : none;
    }
    std::vector<int> clus;  // sorted
    int role = 0;           // 1: scaled rows p1, 2: rows below them p2
    bool alive = true;
  };
  struct RC {
    std::vector<int> slots;
    std::vector<int> groups;
    bool alive = false;
  };

  Handle& H;
  Plan& P;
  // The library's stream.  Converting `st` to hipStream_t first issues the
  // descriptor uploads still pending (upload() below defers and merges
  // them), so every operation enqueued through it runs after its
  // descriptors have been copied.
  struct Stream {
    Factorizer* f;
    operator hipStream_t() const {
      f->flush_uploads();
      return f->raw_st_;
    }
  };
  hipStream_t raw_st_;
  Stream st{this};
  double eps_;
  const int* forced_;
  int nforced_;
  int fpos_ = 0;
  std::vector<RG> G;
  std::vector<RC> C;
  std::set<int> live;
  std::vector<int> pos;
  int level_ = 0, round_ = 0;
  int launches_ = 0, syncs_ = 0;
  double flops_[5] = {0, 0, 0, 0, 0}, bytes_[5] = {0, 0, 0, 0, 0};
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> timers_;

  // ---- helpers ----
  T* talloc(int64_t elems) { return static_cast<T*>(H.arena.alloc(std::max<int64_t>(1, elems) * sizeof(T))); }
  static int64_t pad(int64_t m) { return std::max<int64_t>(8, (m + 7) / 8 * 8); }
  static bool has(const std::vector<int>& v, int c) { return std::binary_search(v.begin(), v.end(), c); }

  // Descriptor upload through pinned staging memory.  The copy is not
  // issued at once: uploads that follow each other in both the staging
  // and the device arena (same 256-byte rounding in both) are merged into
  // one pending copy, issued when anything is next enqueued on `st`.  A
  // pointer returned here must therefore only be handed to work enqueued
  // in a later statement (never in the same argument list as `st`, whose
  // conversion may be evaluated first).
  char* pend_h_ = nullptr;
  char* pend_d_ = nullptr;
  size_t pend_n_ = 0;
  void flush_uploads() {
    if (pend_n_ == 0) return;
    const size_t n = pend_n_;
    pend_n_ = 0;
    SPAQR_HIP(hipMemcpyAsync(pend_d_, pend_h_, n, hipMemcpyHostToDevice, raw_st_));
  }
  template <class D>
  D* upload(const std::vector<D>& v) {
    if (v.empty()) return nullptr;
    const size_t b = v.size() * sizeof(D);
    const size_t br = (b + 255) & ~size_t(255);
    char* hp = static_cast<char*>(H.stage.alloc(br));
    std::memcpy(hp, v.data(), b);
    char* dp = static_cast<char*>(H.arena.alloc(br));
    if (pend_n_ > 0 && hp == pend_h_ + pend_n_ && dp == pend_d_ + pend_n_) {
      pend_n_ += br;
    } else {
      flush_uploads();
      pend_h_ = hp, pend_d_ = dp, pend_n_ = br;
    }
    return reinterpret_cast<D*>(dp);
  }

  // int pool: colmaps etc. collected per launch, uploaded once
  struct IntPool {
    std::vector<int> v;
    size_t add(const std::vector<int>& a) {
      size_t o = v.size();
      v.insert(v.end(), a.begin(), a.end());
      return o;
    }
  };

  // pos[s] = position of slot s in `slots` (until clear_slots)
  void index_slots(const std::vector<int>& slots) {
    for (size_t i = 0; i < slots.size(); ++i) pos[slots[i]] = (int)i;
  }
  void clear_slots(const std::vector<int>& slots) {
    for (int v : slots) pos[v] = -1;
  }
  // out[c] = pos[cols[c]]; false if a slot of cols is not indexed
  bool lookup(const std::vector<int>& cols, int* out) const {
    bool ok = true;
    for (size_t c = 0; c < cols.size(); ++c) {
      out[c] = pos[cols[c]];
      ok = ok && out[c] >= 0;
    }
    return ok;
  }
  // Column maps of front gathers, expanded on the device: the host lists
  // the front column of each of a group's slots, k_expand_maps turns the
  // list into the gather's map (entry c: g's column holding front column c,
  // -1 where g has none).
  struct FrontMaps {
    IntPool fpos;
    std::vector<ExpandDesc> xd;
    std::vector<size_t> fo;
    int64_t dense = 0;
    std::unordered_map<const SlotList*, size_t> cache;  // this front's maps by slot list
  };
  // Records the map of group g into a front of n columns indexed in pos
  // (index_slots of the front's columns); returns its offset in the
  // expanded maps.
  size_t front_map(FrontMaps& fm, const RG& g, int n) {
    // groups sharing a slot list share the map (within one front)
    auto hit = fm.cache.find(g.sl.get());
    if (hit != fm.cache.end()) return hit->second;
    ExpandDesc e{};
    e.nslots = (int)g.slots().size();
    e.n = n;
    fm.fo.push_back(fm.fpos.v.size());
    for (int v : g.slots()) fm.fpos.v.push_back(pos[v]);
    fm.xd.push_back(e);
    const size_t o = (size_t)fm.dense;
    fm.dense += n;
    fm.cache.emplace(g.sl.get(), o);
    return o;
  }
  // Uploads the lists and expands them on the device (in stream order
  // before the gather); returns the expanded maps.
  int* expand(FrontMaps& fm) {
    int* dense = static_cast<int*>(H.arena.alloc(std::max<int64_t>(1, fm.dense) * sizeof(int)));
    int* dp = upload(fm.fpos.v);
    size_t off = 0;
    for (size_t k = 0; k < fm.xd.size(); ++k) {
      fm.xd[k].fpos = dp ? dp + fm.fo[k] : nullptr;
      fm.xd[k].out = dense + off;
      off += fm.xd[k].n;
    }
    const ExpandDesc* dxd = upload(fm.xd);
    launch_expand_maps(dxd, (int)fm.xd.size(), st);
    ++launches_;
    return dense;
  }
  // Appends the required map of an indexed column list (index_slots of the
  // n columns of cluster p) into group g's columns: entry k is g's column
  // holding column k of the list.
  size_t subset_map_from(IntPool& pool, const RG& g, int n, int p) {
    const size_t o = pool.v.size();
    pool.v.resize(o + n, -1);
    int* m = pool.v.data() + o;
    const std::vector<int>& gs = g.slots();
    // first only the blocks of p and of the clusters merged into it (the
    // list is cluster by cluster), then the whole list if that missed any
    int found = 0;
    if (g.sl)
      for (const auto& b : g.sl->blk)
        if (within(b[0], p))
          for (int i = b[1]; i < b[2]; ++i) {
            const int k = pos[gs[i]];
            if (k >= 0 && m[k] < 0) m[k] = i, ++found;
          }
    if (found < n)
      for (size_t i = 0; i < gs.size(); ++i) {
        const int k = pos[gs[i]];
        if (k >= 0) m[k] = (int)i;
      }
    for (int k = 0; k < n; ++k)
      if (m[k] < 0) throw Error(SPAQR_EARG, "internal: group lacks a column of a touched cluster");
    return o;
  }
  // Appends the required map of `cols` into the indexed slot list.
  size_t subset_map(IntPool& pool, const std::vector<int>& cols) {
    const size_t o = pool.v.size();
    pool.v.resize(o + cols.size());
    if (!lookup(cols, pool.v.data() + o)) throw Error(SPAQR_EARG, "internal: group lacks a column of a touched cluster");
    return o;
  }

  std::vector<int> slots_of(const std::vector<int>& clus) {
    std::vector<int> s;
    for (int c : clus) s.insert(s.end(), C[c].slots.begin(), C[c].slots.end());
    return s;
  }

  // Levels that are scaled and sparsified (Section 4: the first leaf-side
  // levels are skipped, and the root has no interfaces left).
  bool sparsified(int m) const { return m >= 2 && m <= P.depth - P.skip; }

  void sync() {
    const double t = now_s();
    SPAQR_HIP(hipStreamSynchronize(st));
    wait_s_ += now_s() - t;
    ++syncs_;
  }
  double wait_s_ = 0.0;
  int report_fallbacks_ = 0;  // pivot-step loops that fell back to a stream read
  // how long the pivot-step loop waits for the report word to advance before
  // reading the live count through the stream: 20 ms, or
  // SPAQR_PQR_REPORT_WAIT_MS (0 takes the stream read at every wait; tests
  // use it to run that path)
  static double report_wait_s() {
    static const double w = [] {
      const char* e = std::getenv("SPAQR_PQR_REPORT_WAIT_MS");
      return e ? std::max(0.0, std::atof(e)) * 1e-3 : 0.02;
    }();
    return w;
  }

  int next_forced() {
    if (!forced_) return -1;
    if (fpos_ >= nforced_) throw Error(SPAQR_EARG, "forced rank list is too short");
    return forced_[fpos_++];
  }

  void timer_begin(int phase) {
    hipEvent_t a, b;
    SPAQR_HIP(hipEventCreate(&a));
    SPAQR_HIP(hipEventCreate(&b));
    SPAQR_HIP(hipEventRecord(a, st));
    timers_.push_back({phase, {a, b}});
  }
  void timer_end() { SPAQR_HIP(hipEventRecord(timers_.back().second.second, st)); }

  void kill_group(int g) { G[g].alive = false; }

  // touch[c]: groups whose cluster list has held c (may be stale; checked
  // on use).  Kept so an interface can be removed from every group that
  // touches it without scanning all groups.
  std::vector<std::vector<int>> touch;
  void note(int g) {
    for (int c : G[g].clus) touch[c].push_back(g);
  }

  std::vector<int> live_groups() {
    std::vector<int> out;
    for (int c : live)
      for (int g : C[c].groups) out.push_back(g);
    return out;
  }
  // Owner and position in the owner's list of every live group (valid while
  // lgen_[g] == gen_, until the structure changes): the order in which a
  // scan of live_groups() meets them is (owner, position).
  std::vector<int> lgen_, lown_, lpos_;
  int gen_ = 0;
  std::vector<int> cstamp_;  // per cluster: set to cgen_ once listed
  int cgen_ = 0;
  // ascending clusters held by the groups of a and b, s excluded
  std::vector<int> cluster_union(int s, const std::vector<int>& a, const std::vector<int>& b) {
    if (cstamp_.size() < P.clusters.size()) cstamp_.assign(P.clusters.size(), 0);
    ++cgen_;
    cstamp_[s] = cgen_;
    std::vector<int> u;
    for (const auto* lst : {&a, &b})
      for (int g : *lst)
        for (int q : G[g].clus)
          if (cstamp_[q] != cgen_) cstamp_[q] = cgen_, u.push_back(q);
    std::sort(u.begin(), u.end());
    return u;
  }
  void index_live_groups() {
    if (lgen_.size() < G.size()) {
      lgen_.resize(G.size(), 0);
      lown_.resize(G.size(), -1);
      lpos_.resize(G.size(), -1);
    }
    ++gen_;
    for (int c : live)
      for (size_t k = 0; k < C[c].groups.size(); ++k) {
        const int g = C[c].groups[k];
        lgen_[g] = gen_;
        lown_[g] = c;
        lpos_[g] = (int)k;
      }
  }
  bool is_live(int g) const { return g < (int)lgen_.size() && lgen_[g] == gen_; }
  bool holds(int g, int s) const {
    const auto& cl = G[g].clus;
    return std::find(cl.begin(), cl.end(), s) != cl.end();
  }
  // Drops from touch[s] the groups that are dead or no longer hold s, and
  // repeated entries, once the list has doubled since it was last compacted.
  std::vector<int> tsize_;
  void compact_touch(int s) {
    auto& t = touch[s];
    if (tsize_.size() < touch.size()) tsize_.resize(touch.size(), 0);
    if (t.size() <= 2 * (size_t)tsize_[s] + 16) return;
    std::sort(t.begin(), t.end());
    t.erase(std::unique(t.begin(), t.end()), t.end());
    t.erase(std::remove_if(t.begin(), t.end(), [&](int g) { return !G[g].alive || !holds(g, s); }), t.end());
    tsize_[s] = (int)t.size();
  }
  // live groups whose cluster list holds s (touch[s] filtered), in the
  // order of a scan of live_groups(); owned by s too unless skip_own
  std::vector<int> holders(int s, bool skip_own) {
    compact_touch(s);
    std::vector<std::pair<int64_t, int>> k;
    for (int g : touch[s]) {
      if (!is_live(g) || (skip_own && lown_[g] == s)) continue;
      if (holds(g, s)) k.emplace_back(((int64_t)lown_[g] << 32) | (uint32_t)lpos_[g], g);
    }
    std::sort(k.begin(), k.end());
    std::vector<int> h;
    h.reserve(k.size());
    for (size_t i = 0; i < k.size(); ++i)
      if (i == 0 || k[i].first != k[i - 1].first) h.push_back(k[i].second);
    return h;
  }

  void record_op(int kind, int phase, const void* R, const void* tau, int64_t ld, int n1, int n2,
                 const std::vector<int>& s1, const std::vector<int>& s2) {
    OpRec o;
    o.kind = kind;
    o.level = level_;
    o.round = round_;
    o.phase = phase;
    o.R = R;
    o.tau = tau;
    o.ld = ld;
    o.n1 = n1;
    o.n2 = n2;
    o.s1 = s1;
    o.s2 = s2;
    H.ops.push_back(std::move(o));
  }

  // Debug hook: with SPAQR_DEBUG_DIR set, every gathered front is written to
  // <dir>/<tag>_L<level>_<key0>_<key1>.bin as int64 m, n; int32 slots[n];
  // double data[m*n] column-major.  Off (and free) otherwise.
  void dump_front(const char* tag, int cluster, const T* F, int64_t ld, int m, int n,
                  const std::vector<int>& cols) {
    static const char* dir = std::getenv("SPAQR_DEBUG_DIR");
    if (!dir) return;
    sync();
    std::vector<T> buf((size_t)ld * std::max(1, n));
    SPAQR_HIP(hipMemcpy(buf.data(), F, buf.size() * sizeof(T), hipMemcpyDeviceToHost));
    const Cluster& c = P.clusters[cluster];
    std::string path = std::string(dir) + "/" + tag + "_L" + std::to_string(level_) + "_" +
                       std::to_string(c.key0) + "_" + std::to_string(c.key1) + ".bin";
    FILE* fp = std::fopen(path.c_str(), "wb");
    if (!fp) return;
    int64_t mn[2] = {m, n};
    std::fwrite(mn, sizeof(int64_t), 2, fp);
    std::vector<int32_t> s(cols.begin(), cols.end());
    std::fwrite(s.data(), sizeof(int32_t), s.size(), fp);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < m; ++i) {
        const double v = (double)buf[(size_t)i + (size_t)j * ld];
        std::fwrite(&v, sizeof(double), 1, fp);
      }
    std::fclose(fp);
  }

  // Debug hook: SPAQR_DEBUG_SHAPES=1 prints one line per batched launch.
  template <class D>
  void log_shapes(const char* what, const std::vector<D>& v) {
    static const bool on = std::getenv("SPAQR_DEBUG_SHAPES") != nullptr;
    if (!on || v.empty()) return;
    int mm = 0, mn = 0;
    double work = 0;
    for (auto& d : v) {
      mm = std::max(mm, d.m);
      mn = std::max(mn, d.n);
      work += (double)d.m * d.n;
    }
    std::fprintf(stderr, "[spaqr] L%d r%d %-8s count %4zu max_m %5d max_n %6d sum_mn %.3e\n", level_, round_,
                 what, v.size(), mm, mn, work);
    static const bool each = on && std::getenv("SPAQR_DEBUG_SHAPES")[0] == '2';
    if (each)
      for (auto& d : v) std::fprintf(stderr, "[spaqr]   %s L%d r%d m %d n %d\n", what, level_, round_, d.m, d.n);
  }

  // grow-only device scratch (valid for the whole factorization)
  double* scratch(std::vector<std::pair<double*, size_t>>& pool, int slot, size_t n) {
    if ((int)pool.size() <= slot) pool.resize(slot + 1, {nullptr, 0});
    auto& e = pool[slot];
    if (n > e.second) {
      e.second = std::max(n, 2 * e.second);
      e.first = static_cast<double*>(H.arena.alloc(e.second * sizeof(double)));
    }
    return e.first;
  }
  std::vector<std::pair<double*, size_t>> qrpool_;

  // Algorithmic work of a rank-revealing-QR batch whose step launches were
  // timed, once its ranks are known: per matrix (m x n, rank r) the flops
  // of a pivoted QR truncated at r, 4mnr - 2r^2(m+n) + 4r^3/3 plus 2mn for
  // the column norms, and its block read once and its kept rows written
  // once, s (mn + rn) bytes; each timed launch (one pivot step of every
  // matrix of the batch) is credited its share, timed / launched.
  void account_pqr(const std::vector<PQRDesc>& q, const int* ranks) {
    if (!H.kt.on("pqr_step") || pqr_launched_ == 0) return;
    const double share = (double)timed_steps_.size() / pqr_launched_;
    for (size_t k = 0; k < q.size(); ++k) {
      const double m = q[k].m, n = q[k].n, r = ranks[k];
      H.kt.flops += share * (4 * m * n * r - 2 * r * r * (m + n) + 4 * r * r * r / 3 + 2 * m * n);
      H.kt.bytes += share * sizeof(T) * (m * n + r * n);
    }
    timed_steps_.clear();
    pqr_launched_ = 0;
  }
  int pqr_launched_ = 0;
  std::vector<int> timed_steps_;

  // After a sync: a persistent pivoted QR that abandoned a wait left ranks of
  // 0 and partial factors; report it.
  // (fetch_pqr_err queues the copy of the flag ahead of that sync)
  int* pqr_err_h_ = nullptr;
  void fetch_pqr_err() {
    if (!pqr_err_h_) pqr_err_h_ = static_cast<int*>(H.stage.alloc(sizeof(int)));
    SPAQR_HIP(hipMemcpyAsync(pqr_err_h_, H.d_pqr_err, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  void check_pqr() {
    if (pqr_err_h_ && *pqr_err_h_) {
      *pqr_err_h_ = 0;
      SPAQR_HIP(hipMemset(H.d_pqr_err, 0, sizeof(int)));
      throw Error(SPAQR_EHIP, "a wait between the work-groups of a kernel exceeded its time limit");
    }
  }

  // Batched rank-revealing QR in one cooperative launch, when the batch
  // qualifies (see pqr_run_width); false otherwise.
  bool run_pqr_persistent(std::vector<PQRDesc>& q, int max_m) {
    std::vector<int> ns;
    ns.reserve(q.size());
    for (const PQRDesc& e : q) ns.push_back(e.n);
    int rows = 0;
    const int cw = pqr_run_width<T>(max_m, ns, &rows);
    if (cw <= 0) return false;
    int total = 0, groups = 0;
    std::vector<int2> bmap;
    for (size_t k = 0; k < q.size(); ++k) {
      q[k].cw = cw;
      q[k].blk0 = total;
      q[k].nblk = std::max(1, (q[k].n + cw - 1) / cw);
      q[k].g0 = groups;
      groups += std::max(1, (q[k].n + 7) / 8);
      for (int c = 0; c < q[k].nblk; ++c) bmap.push_back(make_int2((int)k, c));
      total += q[k].nblk;
    }
    const PQRDesc* d = upload(q);
    const int2* dmap = upload(bmap);
    PQRXch xc{};
    xc.G = total;
    xc.rows = rows;
    const size_t words = pqr_xch_words(total, rows, groups, sizeof(T));
    auto* buf = static_cast<unsigned long long*>(H.arena.alloc(words * sizeof(unsigned long long)));
    SPAQR_HIP(hipMemsetAsync(buf, 0, words * sizeof(unsigned long long), st));
    xc.part = buf;
    xc.pub = buf + 6 * (size_t)total;
    xc.frop = xc.pub + 2 * (size_t)total * rows * (sizeof(T) / 4);
    xc.err = H.d_pqr_err;
    static const bool dbg = std::getenv("SPAQR_DEBUG_PQR") != nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (dbg) {
      SPAQR_HIP(hipEventCreate(&e0));
      SPAQR_HIP(hipEventCreate(&e1));
      SPAQR_HIP(hipEventRecord(e0, st));
    }
    launch_pqr_run<T>(d, total, dmap, xc, eps_, cw, nullptr, st);
    ++launches_;
    if (dbg) {
      SPAQR_HIP(hipEventRecord(e1, st));
      SPAQR_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SPAQR_HIP(hipEventElapsedTime(&ms, e0, e1));
      int rmax = 0;
      for (const PQRDesc& e : q) {
        int r = 0;
        SPAQR_HIP(hipMemcpy(&r, e.rank_out, sizeof(int), hipMemcpyDeviceToHost));
        rmax = std::max(rmax, r);
      }
      std::fprintf(stderr, "[pqr_run] L%d r%d nmat %zu G %d cw %d rows %d max_m %d steps %d  %.1f us  %.2f us/step\n",
                   level_, round_, q.size(), total, cw, rows, max_m, rmax, ms * 1e3, ms * 1e3 / std::max(1, rmax + 1));
      SPAQR_HIP(hipEventDestroy(e0));
      SPAQR_HIP(hipEventDestroy(e1));
    }
    return true;
  }

  // Batched rank-revealing QR: one launch per pivot step until every
  // matrix has stopped (polled every few steps).
  void run_pqr(std::vector<PQRDesc>& q) {
    if (q.empty()) return;
    int total = 0, kmax = 0, max_m = 1, live_m = 0;
    for (const PQRDesc& e : q) max_m = std::max(max_m, e.m);
    if (run_pqr_persistent(q, max_m)) return;
    // 8-column chunks: wider ones (fewer partials to scan, more columns per
    // wave) measured slower at every matrix height here
    const int cw = PQR_CW;
    for (size_t k = 0; k < q.size(); ++k) {
      q[k].cw = cw;
      q[k].blk0 = total;
      q[k].nblk = std::max(1, (q[k].n + cw - 1) / cw);
      total += q[k].nblk;
      kmax = std::max(kmax, std::min(q[k].m, q[k].n));
      max_m = std::max(max_m, q[k].m);
      if (std::min(q[k].m, q[k].n) > 0) ++live_m;
    }
    // Work-groups listed matrix by matrix in decreasing order of min(m, n),
    // the most steps a matrix can take: a matrix has stopped by the end of
    // step min(m, n) (exhausted, if nothing stopped it before) and has copied
    // its final state to both state slots by the end of the step after, so
    // step i launches only the prefix of matrices with min(m, n) >= i - 1.
    // The list order changes nothing computed: each work-group finds its
    // matrix and chunk in the list, and partials keep their per-matrix place.
    std::vector<int> order(q.size());
    for (size_t k = 0; k < q.size(); ++k) order[k] = (int)k;
    auto steps_of = [&](int k) { return std::min(q[k].m, q[k].n); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return steps_of(a) > steps_of(b); });
    std::vector<int2> bmap;
    for (int k : order)
      for (int c = 0; c < q[k].nblk; ++c) bmap.push_back(make_int2(k, c));
    size_t pre_k = 0;  // matrices in the launched prefix for the current step
    int pre_g = 0;     // and their work-groups
    double launched_wg = 0.0;
    const PQRDesc* d = upload(q);
    const int2* dmap = upload(bmap);
    std::vector<PQRDesc> qb;
    qb.reserve(bmap.size());
    for (const int2& b : bmap) qb.push_back(q[b.x]);
    const PQRDesc* dblk = upload(qb);
    int* active = upload(std::vector<int>{live_m});
    auto* states = static_cast<PQRState*>(H.arena.alloc(2 * q.size() * sizeof(PQRState)));
    auto* parts = static_cast<PQRPart*>(H.arena.alloc(2 * (size_t)total * sizeof(PQRPart)));
    auto* frop = static_cast<double*>(H.arena.alloc((size_t)total * sizeof(double)));
    int* h_active = static_cast<int*>(H.stage.alloc(sizeof(int)));
    static const bool dbg = std::getenv("SPAQR_DEBUG_PQR") != nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (dbg) {
      SPAQR_HIP(hipEventCreate(&e0));
      SPAQR_HIP(hipEventCreate(&e1));
      SPAQR_HIP(hipEventRecord(e0, st));
    }
    launch_pqr_init<T>(d, total, states, parts, frop, dmap, st);
    ++launches_;
    int steps = 0;
    timed_steps_.clear();
    pqr_launched_ = 0;
    // Steps are launched ahead of the GPU, at most pqr_poll beyond the last
    // step whose kernel has reported the live-matrix count (the report word
    // in pinned host memory, tagged with this batch), so the stream never
    // drains; once a report shows no live matrix, the steps already queued
    // find every matrix stopped and only carry the state over.  Should the
    // report not advance for a long time (more than 20 ms), the count is
    // read through the stream instead.
    unsigned tag = (++H.pqr_tag) & 0xFFFFFFu;
    if (tag == 0) tag = (++H.pqr_tag) & 0xFFFFFFu;  // 0 is what an unwritten report word holds
    int run_left = 0, run_len = 0;  // timed stretch in progress
    // batches of several matrices skip the fetches of the ones that stopped
    const bool check_first = live_m >= kCheckFirstMats;
    volatile unsigned long long* rep = H.h_pqr_report;
    int reported = -1;  // last step whose kernel has reported
    while (steps < kmax) {
      ++pqr_launched_;
      // Timing (spaqr_time_kernel "pqr_step"): every launch is timed, in
      // stretches of `every` consecutive launches bracketed by HIP events on
      // this stream (two event packets per stretch, not per launch); the
      // first launch of a stretch also stamps its own first start and last
      // end on the GPU clock.
      const bool timing = H.kt.on("pqr_step");
      const bool opens = timing && run_left == 0;
      unsigned long long* stamp = opens ? H.kt.stamp(st) : nullptr;
      if (timing) timed_steps_.push_back(steps);
      if (opens) {
        H.kt.mark(st);
        run_left = H.kt.every;
        run_len = 0;
      }
      if (steps == 0 || steps_of(order[pre_k - 1]) < steps - 1) {
        // (re)form the prefix: every matrix that can still be running
        pre_k = 0, pre_g = 0;
        while (pre_k < order.size() && steps_of(order[pre_k]) >= steps - 1) pre_g += q[order[pre_k++]].nblk;
      }
      launched_wg += pre_g;
      launch_pqr_step<T>(dblk, pre_g, total, states, parts, frop, dmap, active, steps, eps_, max_m, cw,
                         H.tune.pqr_reg_rows, stamp, H.d_pqr_report, tag, check_first, st);
      if (timing) {
        ++run_len;
        if (--run_left == 0) H.kt.close(st, run_len);
      }
      ++launches_;
      ++steps;
      if (steps >= kmax) break;
      bool done = false;
      double t_wait = -1.0;
      const double t_spin = now_s();
      for (;;) {
        const unsigned long long w = *rep;
        if ((unsigned)(w >> 40) == tag) {
          const int s = (int)((w >> 20) & 0xFFFFFu);
          if ((w & 0xFFFFFu) == 0) {
            done = true;
            break;
          }
          if (s > reported) reported = s, t_wait = -1.0;
        }
        if (steps - 1 - reported < H.tune.pqr_poll) break;
        const double t = now_s();
        if (t_wait < 0.0) {
          t_wait = t;
        } else if (t - t_wait > report_wait_s()) {
          SPAQR_HIP(hipMemcpyAsync(h_active, active, sizeof(int), hipMemcpyDeviceToHost, st));
          SPAQR_HIP(hipStreamSynchronize(st));  // counted in the spin's wait below
          ++syncs_;
          ++report_fallbacks_;
          done = *h_active == 0;
          reported = steps - 1;
          break;
        }
      }
      wait_s_ += now_s() - t_spin;
      if (done) break;
    }
    if (run_left > 0) H.kt.close(st, run_len);  // a stretch ends with its batch
    launch_pqr_finish<T>(d, (int)q.size(), states, steps, st);
    ++launches_;
    if (dbg) {
      SPAQR_HIP(hipEventRecord(e1, st));
      SPAQR_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SPAQR_HIP(hipEventElapsedTime(&ms, e0, e1));
      // share of the launched work-group steps that belonged to a live matrix
      double live_wg = 0.0;
      for (const PQRDesc& e : q) {
        int r = 0;
        if (e.rank_out) SPAQR_HIP(hipMemcpy(&r, e.rank_out, sizeof(int), hipMemcpyDeviceToHost));
        live_wg += (double)e.nblk * std::min(r + 1, steps);
      }
      std::fprintf(stderr,
                   "[pqr_steps] L%d r%d nmat %zu G %d cw %d max_m %d steps %d  %.1f us  %.2f us/step  live %.3f"
                   "  launched %.3f\n",
                   level_, round_, q.size(), total, cw, max_m, steps, ms * 1e3, ms * 1e3 / std::max(1, steps),
                   live_wg / std::max(1.0, (double)total * steps), launched_wg / std::max(1.0, (double)total * steps));
      SPAQR_HIP(hipEventDestroy(e0));
      SPAQR_HIP(hipEventDestroy(e1));
    }
  }

  void run_qr(const std::vector<QRDesc>& q) {
    if (q.empty()) return;
    QRDesc* d = upload(q);
    log_shapes("qr", q);
    QRWork ws{};
    qr_work_dims(q, &ws.MS, &ws.MT);
    const size_t nf = q.size();
    ws.tbuf = scratch(qrpool_, 0, nf * QR_NB * QR_NB);
    ws.betas = scratch(qrpool_, 1, nf);
    ws.normp = scratch(qrpool_, 2, nf * ws.MS);
    ws.dp = scratch(qrpool_, 3, 2 * nf * ws.MS * QR_NB);
    ws.gp = scratch(qrpool_, 4, nf * ws.MS * QR_NB * QR_NB);
    ws.wp = scratch(qrpool_, 5, nf * ws.MT * ws.MS * QR_NB * QR_TN);
    ws.w = scratch(qrpool_, 6, nf * ws.MT * QR_NB * QR_TN);
    launch_qr<T>(d, q, ws, st, &launches_, &H.kt, H.tune.tall_coop != 0);
  }

  int* flags_ = nullptr;
  int nflags_ = 0;

  void init_groups();
  void eliminate_level(int m);
  void eliminate_round(const std::vector<int>& sel);
  void scale_all();
  void step1_all();
  void step2_round(const std::vector<int>& sel);
  void vanish(int p);
  void merge(int m);
  void reassign_group_rows(int g);
  void build_apply();
};

template <typename T>
void Factorizer<T>::init_groups() {
  const size_t nc = P.clusters.size();
  C.assign(nc, RC());
  touch.assign(nc, {});
  pos.assign(P.N, -1);
  T* base = talloc(P.init_elems);
  SPAQR_HIP(hipMemsetAsync(base, 0, std::max<int64_t>(1, P.init_elems) * sizeof(T), st));
  launch_scatter_csr<T>(base, H.d_init_dst, H.d_ahat, P.nnz, st);
  launches_ += 2;
  const bool built = H.init_slots.size() == P.init_groups.size();
  if (!built) H.init_slots.assign(P.init_groups.size(), nullptr);
  for (size_t k = 0; k < P.init_groups.size(); ++k) {
    const InitGroup& ig = P.init_groups[k];
    RG g;
    g.owner = ig.owner;
    g.data = base + ig.offset;
    g.ld = ig.ld;
    g.nrows = (int)ig.rows.size();
    if (!built) {
      auto L = std::make_shared<SlotList>();
      for (int c : ig.clus) {
        const auto& cells = P.clusters[c].cells;
        L->blk.push_back({c, (int)L->v.size(), (int)(L->v.size() + cells.size())});
        L->v.insert(L->v.end(), cells.begin(), cells.end());
      }
      H.init_slots[k] = L;
    }
    g.sl = H.init_slots[k];
    g.clus = ig.clus;
    C[ig.owner].groups.push_back((int)G.size());
    G.push_back(std::move(g));
    note((int)G.size() - 1);
  }
  for (int f : P.finest) {
    C[f].slots = P.clusters[f].cells;
    C[f].alive = true;
    live.insert(f);
  }
}

// ---- elimination (Section 2.3) ----------------------------------------------
template <typename T>
void Factorizer<T>::eliminate_level(int m) {
  std::vector<int> pending;
  for (int c : live)
    if (P.nodes[P.clusters[c].sep].level == m) pending.push_back(c);
  round_ = 0;
  if (m == 1 && !pending.empty()) {
    int s = pending[0];
    int rows = 0;
    for (int g : C[s].groups) rows += G[g].nrows;
    H.stats.top_cols = (int)C[s].slots.size();
    H.stats.top_rows = rows;
  }
  std::vector<int> mark(P.clusters.size(), 0);
  if (cstamp_.size() < P.clusters.size()) cstamp_.assign(P.clusters.size(), 0);
  while (!pending.empty()) {
    // neighbours of every pending cluster from the current structure: the
    // clusters touched by any live group that s owns or that touches s
    // (the groups s owns, and the live groups of other owners that hold s)
    // (each cluster once, s excluded; the order does not matter below)
    index_live_groups();
    std::vector<std::vector<int>> nb(pending.size());
    for (size_t i = 0; i < pending.size(); ++i) {
      const int s = pending[i];
      auto& u = nb[i];
      ++cgen_;
      cstamp_[s] = cgen_;
      auto add = [&](int g) {
        for (int q : G[g].clus)
          if (cstamp_[q] != cgen_) cstamp_[q] = cgen_, u.push_back(q);
      };
      for (int g : C[s].groups) add(g);
      compact_touch(s);
      for (int g : touch[s])
        if (is_live(g) && lown_[g] != s && holds(g, s)) add(g);
    }
    // greedy round in id order: s joins unless a cluster already taken is
    // its neighbour or has it as a neighbour (mark[] holds both relations)
    std::vector<int> sel, rest;
    for (size_t i = 0; i < pending.size(); ++i) {
      const int s = pending[i];
      bool ok = !mark[s];
      for (int q : nb[i]) ok = ok && mark[q] != 2;
      if (ok) {
        sel.push_back(s);
        mark[s] = 2;
        for (int q : nb[i])
          if (!mark[q]) mark[q] = 1;
      } else {
        rest.push_back(s);
      }
    }
    for (size_t i = 0; i < pending.size(); ++i) {
      mark[pending[i]] = 0;
      for (int q : nb[i]) mark[q] = 0;
    }
    eliminate_round(sel);
    pending.swap(rest);
    ++round_;
  }
}

template <typename T>
void Factorizer<T>::eliminate_round(const std::vector<int>& sel) {
  struct Front {
    int s;
    std::vector<int> owned, foreign, nb, cols;
    Slots s2;  // columns after the eliminated ones (shared by the groups left)
    int m, n, cs, cN, rs;
    T* F;
    int64_t ld;
  };
  std::vector<Front> fr(sel.size());
  FrontMaps fm;
  std::vector<GatherDesc> gd;
  std::vector<size_t> gd_map;
  std::vector<QRDesc> qd;
  int maxc = 0;
  timer_begin(PH_ELIM);
  // foreign rows of every front in one pass over the live groups (by owner
  // id, then group order): groups of other owners that touch the front
  index_live_groups();
  for (size_t i = 0; i < sel.size(); ++i) fr[i].foreign = holders(sel[i], true);
  for (size_t i = 0; i < sel.size(); ++i) {
    Front& f = fr[i];
    f.s = sel[i];
    f.owned = C[f.s].groups;
    f.nb = cluster_union(f.s, f.owned, f.foreign);
    f.cols = C[f.s].slots;
    std::vector<int> ns = slots_of(f.nb);
    f.cols.insert(f.cols.end(), ns.begin(), ns.end());
    f.cs = (int)C[f.s].slots.size();
    f.n = (int)f.cols.size();
    f.cN = f.n - f.cs;
    f.rs = 0;
    for (int g : f.owned) f.rs += G[g].nrows;
    f.m = f.rs;
    for (int g : f.foreign) f.m += G[g].nrows;
    if (f.rs < f.cs) throw Error(SPAQR_EARG, "internal: cluster with fewer rows than columns");
    f.ld = pad(f.m);
    f.F = talloc(f.ld * f.n);
    int64_t row0 = 0;
    index_slots(f.cols);
    fm.cache.clear();
    for (int pass = 0; pass < 2; ++pass)
      for (int g : pass == 0 ? f.owned : f.foreign) {
        GatherDesc d{};
        d.src = G[g].data;
        d.dst = f.F;
        d.src_ld = G[g].ld;
        d.dst_ld = f.ld;
        d.row0 = row0;
        d.col0 = 0;
        d.nrows = G[g].nrows;
        d.ncols = f.n;
        d.transpose = 0;
        gd_map.push_back(front_map(fm, G[g], f.n));
        gd.push_back(d);
        row0 += G[g].nrows;
      }
    clear_slots(f.cols);
    maxc = std::max(maxc, f.n);
    QRDesc q{};
    q.A = f.F;
    q.tau = talloc(std::max(1, std::min(f.m, f.cs)));
    q.lda = f.ld;
    q.m = f.m;
    q.n = f.n;
    q.k = f.cs;
    qd.push_back(q);
    flops_[PH_ELIM] += qr_flops(f.m, f.cs) + 4.0 * f.m * f.cs * f.cN - 2.0 * f.cs * f.cs * f.cN;
    bytes_[PH_ELIM] += 2.0 * sizeof(T) * f.m * f.n;
  }
  int* dmaps = expand(fm);
  for (size_t i = 0; i < gd.size(); ++i) gd[i].colmap = dmaps + gd_map[i];
  const GatherDesc* dgd = upload(gd);
  launch_gather<T>(dgd, (int)gd.size(), maxc, st);
  ++launches_;
  for (auto& f : fr) dump_front("elim", f.s, f.F, f.ld, f.m, f.n, f.cols);
  run_qr(qd);
  timer_end();

  // factor ops, rows of other owners, rows below the diagonal
  std::vector<PQRDesc> qe;
  std::vector<size_t> ext;
  for (size_t i = 0; i < fr.size(); ++i) {
    Front& f = fr[i];
    f.s2 = make_slots(f.cols, f.cs, -1, f.nb);
    const std::vector<int>& s2 = f.s2->v;
    record_op(0, PH_ELIM, f.F, nullptr, f.ld, f.cs, f.cN, C[f.s].slots, s2);
    int64_t off = f.rs;
    for (int g : f.foreign) {
      RG& gr = G[g];
      gr.data = f.F + off + (int64_t)f.cs * f.ld;
      gr.ld = f.ld;
      gr.sl = f.s2;
      // touch lists: only the clusters g did not hold yet (both lists sorted)
      {
        auto it = gr.clus.begin();
        for (int c : f.nb) {
          while (it != gr.clus.end() && *it < c) ++it;
          if (it == gr.clus.end() || *it != c) touch[c].push_back(g);
        }
      }
      gr.clus = f.nb;
      gr.role = 0;
      off += gr.nrows;
    }
    if (f.cN > 0 && f.rs > f.cs) {
      // rows below the diagonal: compressed by a rank-revealing QR in place,
      // truncated by the eps rule on sparsified levels (the reassign phase
      // of Section 4.2) and exact on the leaf-side levels that are not
      // sparsified (Section 4: those levels skip sparsification)
      PQRDesc q{};
      q.exact = sparsified(level_) ? 0 : 1;
      q.A = f.F + f.cs + (int64_t)f.cs * f.ld;
      q.lda = f.ld;
      q.m = f.rs - f.cs;
      q.n = f.cN;
      q.noise = kNoiseRank * unit_roundoff<T>();
      q.work = static_cast<double*>(H.arena.alloc(3 * std::max(1, q.n) * sizeof(double)));
      q.forced = next_forced();
      qe.push_back(q);
      ext.push_back(i);
    }
    for (int g : f.owned) kill_group(g);
    C[f.s].groups.clear();
    C[f.s].alive = false;
    live.erase(f.s);
  }
  if (qe.empty()) return;
  timer_begin(PH_REASSIGN);
  int* d_rank = static_cast<int*>(H.arena.alloc(qe.size() * sizeof(int)));
  for (size_t e = 0; e < qe.size(); ++e) qe[e].rank_out = d_rank + e;
  log_shapes("reassign", qe);
  run_pqr(qe);
  // owner of each kept row (Section 2.3: maximum-norm heuristic)
  IntPool op;
  std::vector<OwnerDesc> od;
  std::vector<size_t> od_cm, od_off;
  int* d_owner_all = nullptr;
  std::vector<size_t> owner_base;
  size_t nown = 0;
  for (size_t e = 0; e < ext.size(); ++e) {
    Front& f = fr[ext[e]];
    const int k = std::min(f.rs - f.cs, f.cN);
    owner_base.push_back(nown);
    nown += k;
  }
  d_owner_all = static_cast<int*>(H.arena.alloc(std::max<size_t>(1, nown) * sizeof(int)));
  for (size_t e = 0; e < ext.size(); ++e) {
    Front& f = fr[ext[e]];
    OwnerDesc d{};
    d.A = qe[e].A;
    d.lda = f.ld;
    d.nrows = std::min(f.rs - f.cs, f.cN);
    d.nrows_dev = d_rank + e;
    d.ncl = (int)f.nb.size();
    std::vector<int> cm(f.cN);
    std::iota(cm.begin(), cm.end(), 0);
    std::vector<int> off(f.nb.size() + 1, 0);
    for (size_t q = 0; q < f.nb.size(); ++q) off[q + 1] = off[q] + (int)C[f.nb[q]].slots.size();
    od_cm.push_back(op.add(cm));
    od_off.push_back(op.add(off));
    d.owner = d_owner_all + owner_base[e];
    od.push_back(d);
  }
  int* dop = upload(op.v);
  for (size_t e = 0; e < od.size(); ++e) {
    od[e].colmap = dop + od_cm[e];
    od[e].cl_off = dop + od_off[e];
  }
  int od_rows = 0;
  for (const OwnerDesc& o : od) od_rows = std::max(od_rows, o.nrows);
  const OwnerDesc* dod = upload(od);
  launch_owner<T>(dod, (int)od.size(), od_rows, st);
  ++launches_;
  int* h_owner = static_cast<int*>(H.stage.alloc((std::max<size_t>(1, nown) + qe.size()) * sizeof(int)));
  int* h_rank = h_owner + std::max<size_t>(1, nown);
  SPAQR_HIP(hipMemcpyAsync(h_owner, d_owner_all, std::max<size_t>(1, nown) * sizeof(int),
                           hipMemcpyDeviceToHost, st));
  SPAQR_HIP(hipMemcpyAsync(h_rank, d_rank, qe.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  fetch_pqr_err();
  sync();
  check_pqr();
  account_pqr(qe, h_rank);
  // new groups, one per (front, owner), appended in front order
  IntPool rp;
  std::vector<RowCopyDesc> rd;
  std::vector<size_t> rd_rows;
  int maxcols = 0;
  for (size_t e = 0; e < ext.size(); ++e) {
    Front& f = fr[ext[e]];
    const int k = h_rank[e];
    H.ranks.push_back(k);
    const double m = qe[e].m, n = qe[e].n;
    flops_[PH_REASSIGN] += 4 * m * n * k - 2.0 * k * k * (m + n) + 4.0 * k * k * k / 3 + 2 * m * n;
    bytes_[PH_REASSIGN] += sizeof(T) * (2 * m * n);
    std::vector<std::vector<int>> by(f.nb.size());
    for (int r = 0; r < k; ++r) by[h_owner[owner_base[e] + r]].push_back(r);
    for (size_t q = 0; q < f.nb.size(); ++q) {
      if (by[q].empty()) continue;
      RG g;
      g.owner = f.nb[q];
      g.nrows = (int)by[q].size();
      g.ld = pad(g.nrows);
      g.data = talloc(g.ld * f.cN);
      g.sl = f.s2;
      g.clus = f.nb;
      RowCopyDesc d{};
      d.src = qe[e].A;
      d.dst = g.data;
      d.src_ld = f.ld;
      d.dst_ld = g.ld;
      d.nrows = g.nrows;
      d.ncols = f.cN;
      d.tri = 0;
      rd_rows.push_back(rp.add(by[q]));
      rd.push_back(d);
      maxcols = std::max(maxcols, f.cN);
      C[g.owner].groups.push_back((int)G.size());
      G.push_back(std::move(g));
      note((int)G.size() - 1);
    }
  }
  int* drp = upload(rp.v);
  for (size_t i = 0; i < rd.size(); ++i) rd[i].rows = drp + rd_rows[i];
  const RowCopyDesc* drd = upload(rd);
  launch_rowcopy<T>(drd, (int)rd.size(), maxcols, st);
  ++launches_;
  timer_end();
}

// ---- interface scaling (Section 2.4) -----------------------------------------
template <typename T>
void Factorizer<T>::scale_all() {
  timer_begin(PH_SCALE);
  std::vector<int> ifaces(live.begin(), live.end());
  FrontMaps fm;
  std::vector<GatherDesc> gd;
  std::vector<size_t> gd_map;
  std::vector<QRDesc> qd;
  std::vector<ExtractDesc> ed;
  std::vector<T*> Rpp(P.clusters.size(), nullptr);
  int maxc = 0;
  int* d_flags = static_cast<int*>(H.arena.alloc(std::max<size_t>(1, ifaces.size()) * sizeof(int)));
  struct SF {
    int p;
    T* F;
    int64_t ld;
    int m, n, cs;
    std::vector<int> nb, cols;
  };
  std::vector<SF> sf;
  std::vector<double> aspects;
  for (size_t i = 0; i < ifaces.size(); ++i) {
    SF f;
    f.p = ifaces[i];
    f.nb = cluster_union(f.p, C[f.p].groups, {});
    f.cols = C[f.p].slots;
    std::vector<int> ns = slots_of(f.nb);
    f.cols.insert(f.cols.end(), ns.begin(), ns.end());
    f.cs = (int)C[f.p].slots.size();
    f.n = (int)f.cols.size();
    f.m = 0;
    for (int g : C[f.p].groups) f.m += G[g].nrows;
    if (f.m < f.cs) throw Error(SPAQR_EARG, "internal: interface with fewer rows than columns");
    f.ld = pad(f.m);
    f.F = talloc(f.ld * f.n);
    int64_t row0 = 0;
    index_slots(f.cols);
    fm.cache.clear();
    for (int g : C[f.p].groups) {
      GatherDesc d{};
      d.src = G[g].data;
      d.dst = f.F;
      d.src_ld = G[g].ld;
      d.dst_ld = f.ld;
      d.row0 = row0;
      d.nrows = G[g].nrows;
      d.ncols = f.n;
      gd_map.push_back(front_map(fm, G[g], f.n));
      gd.push_back(d);
      row0 += G[g].nrows;
    }
    clear_slots(f.cols);
    maxc = std::max(maxc, f.n);
    QRDesc q{};
    q.A = f.F;
    q.tau = talloc(f.cs);
    q.lda = f.ld;
    q.m = f.m;
    q.n = f.n;
    q.k = f.cs;
    qd.push_back(q);
    T* R = talloc((int64_t)f.cs * f.cs);
    Rpp[f.p] = R;
    ExtractDesc e{};
    e.A = f.F;
    e.R = R;
    e.flag = d_flags + i;
    e.lda = f.ld;
    e.ldr = f.cs;
    e.c = f.cs;
    ed.push_back(e);
    aspects.push_back((double)f.m / f.cs);
    if (level_ > 0 && level_ < SPAQR_MAX_LEVELS) {
      H.stats.level_interfaces[level_] += 1;
      H.stats.level_cols[level_] += f.cs;
    }
    flops_[PH_SCALE] += qr_flops(f.m, f.cs) + 4.0 * f.m * f.cs * (f.n - f.cs) - 2.0 * f.cs * f.cs * (f.n - f.cs);
    bytes_[PH_SCALE] += 2.0 * sizeof(T) * f.m * f.n;
    sf.push_back(std::move(f));
  }
  int* dmaps = expand(fm);
  for (size_t i = 0; i < gd.size(); ++i) gd[i].colmap = dmaps + gd_map[i];
  const GatherDesc* dgd = upload(gd);
  launch_gather<T>(dgd, (int)gd.size(), maxc, st);
  ++launches_;
  for (auto& f : sf) dump_front("scale", f.p, f.F, f.ld, f.m, f.n, f.cols);
  run_qr(qd);
  const ExtractDesc* ded = upload(ed);
  launch_extract<T>(ded, (int)ed.size(), st);
  ++launches_;
  for (auto& f : sf) {
    record_op(1, PH_SCALE, Rpp[f.p], nullptr, f.cs, f.cs, 0, C[f.p].slots, {});
    for (int g : C[f.p].groups) kill_group(g);
    C[f.p].groups.clear();
    RG p1;
    p1.owner = f.p;
    p1.data = f.F;
    p1.ld = f.ld;
    p1.nrows = f.cs;
    p1.sl = make_slots(f.cols, 0, f.p, f.nb);
    p1.clus = f.nb;
    p1.clus.insert(std::lower_bound(p1.clus.begin(), p1.clus.end(), f.p), f.p);
    p1.role = 1;
    C[f.p].groups.push_back((int)G.size());
    G.push_back(std::move(p1));
    note((int)G.size() - 1);
    if (f.m > f.cs && f.n > f.cs) {
      RG p2;
      p2.owner = f.p;
      p2.data = f.F + f.cs + (int64_t)f.cs * f.ld;
      p2.ld = f.ld;
      p2.nrows = f.m - f.cs;
      p2.sl = make_slots(f.cols, f.cs, -1, f.nb);
      p2.clus = f.nb;
      p2.role = 2;
      C[f.p].groups.push_back((int)G.size());
      G.push_back(std::move(p2));
      note((int)G.size() - 1);
    }
  }
  // right scaling of every column block by R_qq^-1
  IntPool tp;
  std::vector<TrsmDesc> td;
  std::vector<size_t> td_map;
  int td_rows = 0, td_c = 0;
  for (int g : live_groups()) {
    RG& gr = G[g];
    index_slots(gr.slots());
    for (int q : gr.clus) {
      if (gr.role == 1 && gr.owner == q) continue;
      TrsmDesc d{};
      d.B = gr.data;
      d.R = Rpp[q];
      d.ldb = gr.ld;
      d.ldr = (int64_t)C[q].slots.size();
      d.nrows = gr.nrows;
      d.c = (int)C[q].slots.size();
      td_map.push_back(subset_map(tp, C[q].slots));
      td.push_back(d);
      td_rows = std::max(td_rows, d.nrows);
      td_c = std::max(td_c, d.c);
      flops_[PH_SCALE] += (double)gr.nrows * d.c * d.c;
      bytes_[PH_SCALE] += 2.0 * sizeof(T) * gr.nrows * d.c;
    }
    clear_slots(gr.slots());
  }
  int* dtp = upload(tp.v);
  for (size_t i = 0; i < td.size(); ++i) td[i].colmap = dtp + td_map[i];
  std::vector<int2> trb;
  for (size_t i = 0; i < td.size(); ++i)
    for (int b = 0; b * TRSM_ROWS < td[i].nrows; ++b) trb.push_back(make_int2((int)i, b));
  {
    static const bool on = std::getenv("SPAQR_DEBUG_SHAPES") != nullptr;
    if (on) {
      double work = 0.0, wmax = 0.0;
      int64_t rb = 0;
      for (const TrsmDesc& d : td) {
        rb += (d.nrows + TRSM_ROWS - 1) / TRSM_ROWS;
        work += (double)d.nrows * d.c * d.c;
        wmax = std::max(wmax, (double)d.c * d.c);
      }
      std::fprintf(stderr, "[spaqr] L%d trsm count %zu rowblocks %lld max_rows %d max_c %d sum_rc2 %.3e max_c2 %.3e\n",
                   level_, td.size(), (long long)rb, td_rows, td_c, work, wmax);
    }
  }
  const TrsmDesc* dtd = upload(td);
  const int2* dtrb = upload(trb);
  launch_trsm<T>(dtd, (int)td.size(), td_rows, td_c, dtrb, (int)trb.size(), st);
  ++launches_;
  timer_end();
  // median aspect ratio of the scaled diagonal blocks (Section 4.2)
  if (!aspects.empty() && level_ > 0 && level_ < SPAQR_MAX_LEVELS) {
    std::sort(aspects.begin(), aspects.end());
    const size_t k = aspects.size();
    H.stats.level_aspect[level_] = k % 2 ? aspects[k / 2] : 0.5 * (aspects[k / 2 - 1] + aspects[k / 2]);
  }
  // rank-deficiency flags are read together with the step-1 ranks
  flags_ = d_flags;
  nflags_ = (int)ifaces.size();
}

// ---- sparsification step 1 (Section 2.5.1) -----------------------------------
template <typename T>
void Factorizer<T>::step1_all() {
  timer_begin(PH_SPARSIFY);
  std::vector<int> who;
  for (int p : live)
    for (int g : C[p].groups)
      if (G[g].role == 2) who.push_back(g);
  int* d_rank = static_cast<int*>(H.arena.alloc(std::max<size_t>(1, who.size()) * sizeof(int)));
  std::vector<PQRDesc> pd;
  for (size_t i = 0; i < who.size(); ++i) {
    RG& gr = G[who[i]];
    PQRDesc d{};
    d.A = gr.data;
    d.n = (int)gr.slots().size();
    d.m = gr.nrows;
    d.lda = gr.ld;
    d.work = static_cast<double*>(H.arena.alloc(3 * std::max(1, d.n) * sizeof(double)));
    d.rank_out = d_rank + i;
    d.forced = next_forced();
    d.noise = kNoiseRank * unit_roundoff<T>();
    pd.push_back(d);
  }
  log_shapes("step1", pd);
  run_pqr(pd);
  const size_t nr = std::max<size_t>(1, who.size());
  int* h = static_cast<int*>(H.stage.alloc((nr + nflags_ + 1) * sizeof(int)));
  SPAQR_HIP(hipMemcpyAsync(h, d_rank, nr * sizeof(int), hipMemcpyDeviceToHost, st));
  if (nflags_ > 0)
    SPAQR_HIP(hipMemcpyAsync(h + nr, flags_, nflags_ * sizeof(int), hipMemcpyDeviceToHost, st));
  fetch_pqr_err();
  sync();
  check_pqr();
  for (int i = 0; i < nflags_; ++i)
    if (h[nr + i]) throw Error(SPAQR_ERANK, "a scaling block is numerically rank deficient");
  account_pqr(pd, h);
  for (size_t i = 0; i < who.size(); ++i) {
    const int r = h[i];
    RG& gr = G[who[i]];
    H.ranks.push_back(r);
    if (level_ > 0 && level_ < SPAQR_MAX_LEVELS) H.stats.level_rank1[level_] += r;
    const double m = gr.nrows, n = (double)gr.slots().size();
    flops_[PH_SPARSIFY] += 4 * m * n * r - 2.0 * r * r * (m + n) + 4.0 * r * r * r / 3 + 2 * m * n;
    bytes_[PH_SPARSIFY] += sizeof(T) * (2 * m * n);
    gr.nrows = r;
    if (r == 0) {
      auto& lst = C[gr.owner].groups;
      lst.erase(std::remove(lst.begin(), lst.end(), who[i]), lst.end());
      kill_group(who[i]);
    }
  }
  timer_end();
}

// ---- sparsification step 2 (Section 2.5.2) -----------------------------------
template <typename T>
void Factorizer<T>::step2_round(const std::vector<int>& sel) {
  timer_begin(PH_SPARSIFY);
  struct S2 {
    int p, p1, cp, K;
    std::vector<int> blocks, others, oslots, pslots;
    T* Cb;
    int64_t ldc;
    T* V;
    T* tau;
  };
  std::vector<S2> ss(sel.size());
  IntPool pool;
  std::vector<GatherDesc> gd;
  std::vector<size_t> gd_map;
  std::vector<PQRDesc> pd;
  std::vector<ScatterDesc> sd;
  std::vector<size_t> sd_map;
  int* d_rank = static_cast<int*>(H.arena.alloc(std::max<size_t>(1, sel.size()) * sizeof(int)));
  int maxc = 0;
  // every live group touching p, except p's scaled rows, in live-group order
  {
    std::vector<int> sidx(P.clusters.size(), -1);
    for (size_t i = 0; i < sel.size(); ++i) {
      sidx[sel[i]] = (int)i;
      ss[i].p1 = -1;
      for (int g : C[sel[i]].groups)
        if (G[g].role == 1) ss[i].p1 = g;
      if (ss[i].p1 < 0) throw Error(SPAQR_EARG, "internal: interface without scaled rows");
    }
    index_live_groups();
    for (size_t i = 0; i < sel.size(); ++i)
      for (int g : holders(sel[i], false))
        if (g != ss[i].p1) ss[i].blocks.push_back(g);
  }
  for (size_t i = 0; i < sel.size(); ++i) {
    S2& s = ss[i];
    s.p = sel[i];
    for (int c : G[s.p1].clus)
      if (c != s.p) s.others.push_back(c);
    s.oslots = slots_of(s.others);
    s.pslots = C[s.p].slots;
    s.cp = (int)s.pslots.size();
    s.K = (int)s.oslots.size();
    for (int g : s.blocks) s.K += G[g].nrows;
    s.ldc = pad(s.cp);
    s.Cb = talloc(s.ldc * std::max(1, s.K));
    s.V = talloc((int64_t)s.cp * std::max(1, std::min(s.cp, s.K)));
    s.tau = talloc(std::max(1, std::min(s.cp, s.K)));
    int64_t col0 = 0;
    index_slots(s.pslots);
    std::unordered_map<const SlotList*, size_t> bcache;  // blocks sharing a slot list share the map
    for (int g : s.blocks) {
      auto hit = bcache.find(G[g].sl.get());
      const size_t o = hit != bcache.end() ? hit->second : subset_map_from(pool, G[g], s.cp, s.p);
      bcache.emplace(G[g].sl.get(), o);
      GatherDesc d{};
      d.src = G[g].data;
      d.dst = s.Cb;
      d.src_ld = G[g].ld;
      d.dst_ld = s.ldc;
      d.row0 = 0;
      d.col0 = col0;
      d.nrows = G[g].nrows;
      d.ncols = s.cp;
      d.transpose = 1;
      gd_map.push_back(o);
      gd.push_back(d);
      ScatterDesc w{};
      w.C = s.Cb;
      w.dst = G[g].data;
      w.rank = d_rank + i;
      w.ldc = s.ldc;
      w.ld = G[g].ld;
      w.col0 = col0;
      w.nrows = G[g].nrows;
      w.ncols = s.cp;
      w.transpose = 1;
      sd_map.push_back(o);
      sd.push_back(w);
      col0 += G[g].nrows;
    }
    clear_slots(s.pslots);
    {
      index_slots(G[s.p1].slots());
      const size_t o = subset_map(pool, s.oslots);
      const size_t oi = subset_map(pool, s.pslots);
      clear_slots(G[s.p1].slots());
      GatherDesc d{};
      d.src = G[s.p1].data;
      d.dst = s.Cb;
      d.src_ld = G[s.p1].ld;
      d.dst_ld = s.ldc;
      d.row0 = 0;
      d.col0 = col0;
      d.nrows = s.cp;
      d.ncols = (int)s.oslots.size();
      gd_map.push_back(o);
      gd.push_back(d);
      ScatterDesc w{};
      w.C = s.Cb;
      w.dst = G[s.p1].data;
      w.rank = d_rank + i;
      w.ldc = s.ldc;
      w.ld = G[s.p1].ld;
      w.col0 = col0;
      w.nrows = s.cp;
      w.ncols = (int)s.oslots.size();
      sd_map.push_back(o);
      sd.push_back(w);
      ScatterDesc idw{};
      idw.dst = G[s.p1].data;
      idw.rank = d_rank + i;
      idw.ld = G[s.p1].ld;
      idw.identity = 1;
      sd_map.push_back(oi);
      sd.push_back(idw);
    }
    maxc = std::max(maxc, std::max(s.cp, (int)s.oslots.size()));
    PQRDesc q{};
    q.A = s.Cb;
    q.V = s.V;
    q.tau = s.tau;
    q.lda = s.ldc;
    q.m = s.cp;
    q.n = s.K;
    q.work = static_cast<double*>(H.arena.alloc(3 * std::max(1, s.K) * sizeof(double)));
    q.rank_out = d_rank + i;
    q.forced = next_forced();
    q.noise = kNoiseRank * unit_roundoff<T>();
    pd.push_back(q);
  }
  int* dpool = upload(pool.v);
  for (size_t i = 0; i < gd.size(); ++i) gd[i].colmap = dpool + gd_map[i];
  for (size_t i = 0; i < sd.size(); ++i) sd[i].colmap = dpool + sd_map[i];
  const GatherDesc* dgd = upload(gd);
  launch_gather<T>(dgd, (int)gd.size(), maxc, st);
  log_shapes("step2", pd);
  run_pqr(pd);
  const ScatterDesc* dsd = upload(sd);
  launch_scatter<T>(dsd, (int)sd.size(), st);
  launches_ += 2;
  int* h = static_cast<int*>(H.stage.alloc(std::max<size_t>(1, sel.size()) * sizeof(int)));
  SPAQR_HIP(hipMemcpyAsync(h, d_rank, sel.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  fetch_pqr_err();
  sync();
  check_pqr();
  account_pqr(pd, h);
  timer_end();
  for (size_t i = 0; i < ss.size(); ++i) {
    S2& s = ss[i];
    const int r = h[i];
    H.ranks.push_back(r);
    if (level_ > 0 && level_ < SPAQR_MAX_LEVELS) H.stats.level_rank2[level_] += r;
    const double m = s.cp, n = s.K;
    flops_[PH_SPARSIFY] += 4 * m * n * r - 2.0 * r * r * (m + n) + 4.0 * r * r * r / 3 + 2 * m * n;
    bytes_[PH_SPARSIFY] += sizeof(T) * (2 * m * n);
    record_op(2, PH_SPARSIFY, s.V, s.tau, s.cp, s.cp, r, s.pslots, {});
    G[s.p1].nrows = r;
    C[s.p].slots.resize(r);
    if (r == 0) vanish(s.p);
  }
}

// An interface left without coarse columns: its rows move to the cluster
// holding most of their squared norm (the rule of Section 2.3).
template <typename T>
void Factorizer<T>::vanish(int p) {
  C[p].alive = false;
  live.erase(p);
  for (int g : touch[p]) {
    auto& cl = G[g].clus;
    auto it = std::lower_bound(cl.begin(), cl.end(), p);
    if (it != cl.end() && *it == p) cl.erase(it);
  }
  touch[p].clear();
  std::vector<int> mine = C[p].groups;
  C[p].groups.clear();
  for (int g : mine) {
    if (G[g].role == 1 || G[g].nrows == 0) {
      kill_group(g);
      continue;
    }
    auto& cl = G[g].clus;
    cl.erase(std::remove(cl.begin(), cl.end(), p), cl.end());
    reassign_group_rows(g);
  }
}

template <typename T>
void Factorizer<T>::reassign_group_rows(int gi) {
  RG src = G[gi];
  kill_group(gi);
  if (src.clus.empty() || src.nrows == 0) return;
  std::vector<int> off{0};
  IntPool pool;
  index_slots(src.slots());
  for (int c : src.clus) {
    subset_map(pool, C[c].slots);
    off.push_back((int)pool.v.size());
  }
  clear_slots(src.slots());
  const size_t ocm = 0, oof = pool.add(off);
  int* dp = upload(pool.v);
  int* d_owner = static_cast<int*>(H.arena.alloc(src.nrows * sizeof(int)));
  OwnerDesc d{};
  d.A = src.data;
  d.colmap = dp + ocm;
  d.cl_off = dp + oof;
  d.owner = d_owner;
  d.lda = src.ld;
  d.nrows = src.nrows;
  d.ncl = (int)src.clus.size();
  const OwnerDesc* dod = upload(std::vector<OwnerDesc>{d});
  launch_owner<T>(dod, 1, d.nrows, st);
  int* h = static_cast<int*>(H.stage.alloc(src.nrows * sizeof(int)));
  SPAQR_HIP(hipMemcpyAsync(h, d_owner, src.nrows * sizeof(int), hipMemcpyDeviceToHost, st));
  sync();
  std::vector<std::vector<int>> by(src.clus.size());
  for (int r = 0; r < src.nrows; ++r) by[h[r]].push_back(r);
  IntPool rp;
  std::vector<RowCopyDesc> rd;
  std::vector<size_t> rmap;
  for (size_t q = 0; q < by.size(); ++q) {
    if (by[q].empty()) continue;
    RG g;
    g.owner = src.clus[q];
    g.nrows = (int)by[q].size();
    g.ld = pad(g.nrows);
    g.data = talloc(g.ld * (int64_t)src.slots().size());
    g.sl = src.sl;
    g.clus = src.clus;
    RowCopyDesc c{};
    c.src = src.data;
    c.dst = g.data;
    c.src_ld = src.ld;
    c.dst_ld = g.ld;
    c.nrows = g.nrows;
    c.ncols = (int)src.slots().size();
    rmap.push_back(rp.add(by[q]));
    rd.push_back(c);
    C[g.owner].groups.push_back((int)G.size());
    G.push_back(std::move(g));
    note((int)G.size() - 1);
  }
  int* drp = upload(rp.v);
  for (size_t i = 0; i < rd.size(); ++i) rd[i].rows = drp + rmap[i];
  const RowCopyDesc* drd = upload(rd);
  launch_rowcopy<T>(drd, (int)rd.size(), (int)src.slots().size(), st);
  launches_ += 2;
}

// ---- merge (Section 2.6) ------------------------------------------------------
template <typename T>
void Factorizer<T>::merge(int m) {
  std::vector<int> remap(P.clusters.size(), -1);
  bool any = false;
  for (const NDNode& S : P.nodes) {
    if (S.leaf() || S.level >= m) continue;
    const int fin = std::max(S.level, P.depth - 1);
    const int cur = std::min(std::max(S.level, m - 1), fin);
    const int tgt = std::min(std::max(S.level, m - 2), fin);
    if (tgt >= cur) continue;
    for (int pc : S.pieces[tgt - S.level]) {
      RC& par = C[pc];
      par.slots.clear();
      par.groups.clear();
      for (int k : P.clusters[pc].children) {
        if (!C[k].alive) continue;
        par.slots.insert(par.slots.end(), C[k].slots.begin(), C[k].slots.end());
        for (int g : C[k].groups) {
          G[g].owner = pc;
          par.groups.push_back(g);
        }
        C[k].groups.clear();
        C[k].alive = false;
        live.erase(k);
        remap[k] = pc;
        any = true;
      }
      par.alive = !par.slots.empty();
      if (par.alive) live.insert(pc);
    }
  }
  if (!any) return;
  for (int g : live_groups()) {
    auto& cl = G[g].clus;
    bool hit = false;
    for (int& c : cl)
      if (remap[c] >= 0) {
        c = remap[c], hit = true;
        touch[c].push_back(g);  // the other clusters' lists hold g already
      }
    if (!hit) continue;
    std::sort(cl.begin(), cl.end());
    cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
  }
}

// ---- device op lists for the apply sweeps ------------------------------------
template <typename T>
void Factorizer<T>::build_apply() {
  H.batches.clear();
  // Batches of the W sweeps.  Only slot overlap orders the ops here: an op
  // goes to the batch after every earlier op that wrote one of its slots
  // (s1, or an eliminated cluster's neighbours s2) and after every earlier
  // elimination that had one of its own slots s1 as a neighbour.  Two
  // eliminations may share neighbours (their updates are summed per slot).
  // Ops inside a batch touch disjoint slots otherwise, so they commute, and
  // W^-1 / W^-T apply the batches backward / forward.
  std::vector<int> last_w(P.N, -1), last_n(P.N, -1);
  std::vector<std::vector<int>> groups;
  for (size_t k = 0; k < H.ops.size(); ++k) {
    const OpRec& o = H.ops[k];
    int b = 0;
    for (int t : o.s1) b = std::max(b, std::max(last_w[t], last_n[t]) + 1);
    for (int t : o.s2) b = std::max(b, last_w[t] + 1);
    for (int t : o.s1) last_w[t] = std::max(last_w[t], b);
    for (int t : o.s2) last_n[t] = std::max(last_n[t], b);
    if ((int)groups.size() <= b) groups.resize(b + 1);
    groups[b].push_back((int)k);
  }
  int64_t max_stage = 0, max_work = 0;
  for (const std::vector<int>& grp : groups) {
    IntPool pool;
    std::vector<size_t> o1, o2;
    for (int k : grp) {
      o1.push_back(pool.add(H.ops[k].s1));
      o2.push_back(pool.add(H.ops[k].s2));
    }
    int* dp = upload(pool.v);
    std::vector<ApplyOp> ao;
    int mx = 0;
    double bytes = 0.0, flops = 0.0;
    // neighbour contributions of the eliminations (W^-T): staging offsets
    // per op, and per touched slot the list of offsets in op order
    int nstage = 0;
    int64_t pw = 0;
    std::vector<int2> chunks;
    std::vector<std::pair<int, int>> contrib;  // (slot, staging offset), op order within a slot
    for (size_t gi = 0; gi < grp.size(); ++gi) {
      OpRec& o = H.ops[grp[gi]];
      o.d_s1 = dp + o1[gi];
      o.d_s2 = dp + o2[gi];
      ApplyOp a{};
      a.R = o.R;
      a.tau = o.tau;
      a.s1 = o.d_s1;
      a.s2 = o.d_s2;
      a.ld = o.ld;
      a.n1 = o.n1;
      a.n2 = o.n2;
      a.kind = o.kind;
      a.nstage = 0;
      a.poff = 0;
      a.nchunk = 0;
      if (o.kind == 0 && o.n1 > 0 && o.n2 > 0) {
        a.nstage = nstage;
        for (int c = 0; c < o.n2; ++c) contrib.push_back({o.s2[c], nstage + c});
        nstage += o.n2;
        a.nchunk = (o.n2 + APPLY_CHUNK - 1) / APPLY_CHUNK;
        a.poff = pw;
        pw += (int64_t)o.n1 * a.nchunk;
        for (int k = 0; k < a.nchunk; ++k) chunks.push_back(make_int2((int)ao.size(), k));
      }
      ao.push_back(a);
      mx = std::max(mx, o.n1);
      // algorithmic traffic: factor entries once, vector slots read + written
      const double n1 = o.n1, n2 = o.n2;
      const double entries = o.kind == 0 ? n1 * (n1 + 1) / 2 + n1 * n2 : (o.kind == 1 ? n1 * (n1 + 1) / 2 : n1 * n2);
      bytes += sizeof(T) * entries + 8.0 * (2 * n1 + (o.kind == 0 ? 2 * n2 : 0)) + 4.0 * (n1 + n2);
      flops += 2.0 * entries;
    }
    ApplyBatch b;
    b.bytes = bytes;
    b.flops = flops;
    b.d_ops = upload(ao);
    b.n = (int)ao.size();
    b.max_n1 = mx;
    if (!chunks.empty()) {
      b.d_chunks = upload(chunks);
      b.nchunks = (int)chunks.size();
      max_work = std::max(max_work, pw);
    }
    if (!contrib.empty()) {
      std::stable_sort(contrib.begin(), contrib.end(),
                       [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
      std::vector<int> ns, np{0}, no;
      for (size_t e = 0; e < contrib.size(); ++e) {
        if (e == 0 || contrib[e].first != contrib[e - 1].first) {
          if (e) np.push_back((int)e);
          ns.push_back(contrib[e].first);
        }
        no.push_back(contrib[e].second);
      }
      np.push_back((int)contrib.size());
      b.d_nslots = upload(ns);
      b.d_nptr = upload(np);
      b.d_noff = upload(no);
      b.n_nslots = (int)ns.size();
      max_stage = std::max<int64_t>(max_stage, nstage);
    }
    H.batches.push_back(b);
  }
  H.d_nstage = max_stage > 0 ? static_cast<double*>(H.arena.alloc(max_stage * sizeof(double))) : nullptr;
  H.d_awork = max_work > 0 ? static_cast<double*>(H.arena.alloc(max_work * sizeof(double))) : nullptr;
  H.nstage_elems = max_stage;
  H.awork_elems = max_work;
  // launch arguments of the W sweeps (FNV-1a over pointers and sizes)
  uint64_t key = 1469598103934665603ull;
  auto mix = [&key](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      key ^= (v >> (8 * b)) & 0xff;
      key *= 1099511628211ull;
    }
  };
  mix(H.precision);
  mix((uint64_t)(uintptr_t)H.d_nstage);
  mix((uint64_t)(uintptr_t)H.d_awork);
  for (const ApplyBatch& b : H.batches) {
    mix((uint64_t)(uintptr_t)b.d_ops);
    mix((uint64_t)b.n);
    mix((uint64_t)b.max_n1);
    mix((uint64_t)(uintptr_t)b.d_nslots);
    mix((uint64_t)(uintptr_t)b.d_nptr);
    mix((uint64_t)(uintptr_t)b.d_noff);
    mix((uint64_t)b.n_nslots);
    mix((uint64_t)(uintptr_t)b.d_chunks);
    mix((uint64_t)b.nchunks);
  }
  H.apply_key = key;
}

template <typename T>
void Factorizer<T>::run() {
  const double t0 = now_s();
  init_groups();
  double merge_s = 0.0;
  for (int m = P.depth; m >= 1; --m) {
    level_ = m;
    eliminate_level(m);
    if (sparsified(m) && !live.empty()) {
      scale_all();
      step1_all();
      std::vector<int> pending(live.begin(), live.end());
      std::vector<char> taken(P.clusters.size(), 0), blocked(P.clusters.size(), 0);
      round_ = 0;
      while (!pending.empty()) {
        auto p1 = [&](int p) {
          for (int g : C[p].groups)
            if (G[g].role == 1) return g;
          throw Error(SPAQR_EARG, "internal: interface without scaled rows");
        };
        // p joins unless a taken q lies among the columns of p's scaled
        // rows (taken[q]) or p among q's (blocked[p])
        std::vector<int> sel, rest;
        for (int p : pending) {
          const auto& cl = G[p1(p)].clus;
          bool ok = !blocked[p];
          for (int q : cl) ok = ok && !taken[q];
          if (ok) {
            sel.push_back(p);
            taken[p] = 1;
            for (int q : cl) blocked[q] = 1;
          } else {
            rest.push_back(p);
          }
        }
        for (int p : sel) {
          taken[p] = 0;
          for (int q : G[p1(p)].clus) blocked[q] = 0;
        }
        step2_round(sel);
        pending.swap(rest);
        ++round_;
      }
    }
    const double tm = now_s();
    merge(m);
    merge_s += now_s() - tm;
  }
  if (!live.empty()) throw Error(SPAQR_EARG, "internal: clusters left after the root level");
  if (forced_ && fpos_ != nforced_) throw Error(SPAQR_EARG, "forced rank list not fully used");
  build_apply();
  fetch_pqr_err();
  sync();
  check_pqr();
  H.kt.harvest();
  double ph[5] = {0, 0, 0, 0, merge_s};
  for (auto& t : timers_) {
    float ms = 0.f;
    SPAQR_HIP(hipEventElapsedTime(&ms, t.second.first, t.second.second));
    ph[t.first] += ms * 1e-3;
    (void)hipEventDestroy(t.second.first);
    (void)hipEventDestroy(t.second.second);
  }
  timers_.clear();
  spaqr_stats& S = H.stats;
  S.levels = P.depth;
  S.num_ops = (int)H.ops.size();
  S.num_ranks = (int)H.ranks.size();
  S.launches = launches_;
  S.syncs = syncs_;
  S.sync_wait_seconds = wait_s_;
  int64_t mem = 0;
  for (auto& o : H.ops) {
    if (o.kind == 0)
      mem += (int64_t)o.n1 * (o.n1 + 1) / 2 + (int64_t)o.n1 * o.n2;
    else if (o.kind == 1)
      mem += (int64_t)o.n1 * (o.n1 + 1) / 2;
    else
      mem += (int64_t)o.n1 * o.n2;
  }
  S.mem_factor = mem;
  S.device_bytes = (int64_t)(H.arena.capacity() + H.plan_bytes);
  for (int k = 0; k < 5; ++k) {
    S.flops[k] = flops_[k];
    S.bytes[k] = bytes_[k];
    S.phase_seconds[k] = ph[k];
  }
  S.factor_seconds = now_s() - t0;
}

}  // namespace

// ---------------------------------------------------------------------------
// entry points used by the C-ABI
// ---------------------------------------------------------------------------

void factorize(Handle& H, double eps, const int* forced, int nforced) {
  if (!(eps >= 0.0)) throw Error(SPAQR_EARG, "eps must be >= 0");
  H.ensure_device();
  H.factored = false;
  ++H.factor_gen;
  SPAQR_HIP(hipStreamSynchronize(H.stream));
  H.arena.reset();
  H.kt.used = 0;
  H.stage.reset();
  H.ops.clear();
  H.batches.clear();
  H.ranks.clear();
  const int top_cols = 0;
  H.stats = spaqr_stats{};
  H.stats.top_cols = top_cols;
  H.precision = H.opt.precision;
  if (H.precision == SPAQR_FP32_FACTOR)
    Factorizer<float>(H, eps, forced, nforced).run();
  else
    Factorizer<double>(H, eps, forced, nforced).run();
  H.factored = true;
}

void apply_op_stream(Handle& H, bool transpose, double* x, double* stage, double* work, bool timing,
                     hipStream_t st) {
  if (!stage) stage = H.d_nstage;
  if (!work) work = H.d_awork;
  const int nb = (int)H.batches.size();
  for (int k = 0; k < nb; ++k) {
    const ApplyBatch& b = H.batches[transpose ? k : nb - 1 - k];
    const bool timed = timing && H.kt.pick("apply");
    if (timed) H.kt.mark(st);
    const bool f32 = H.precision == SPAQR_FP32_FACTOR;
    if (!transpose && b.nchunks > 0) {
      if (f32)
        launch_apply_gemv<float>(b.d_ops, b.d_chunks, b.nchunks, false, x, stage, work, st);
      else
        launch_apply_gemv<double>(b.d_ops, b.d_chunks, b.nchunks, false, x, stage, work, st);
    }
    if (f32)
      launch_apply_batch<float>(b.d_ops, b.n, b.max_n1, transpose, x, stage, work, st);
    else
      launch_apply_batch<double>(b.d_ops, b.n, b.max_n1, transpose, x, stage, work, st);
    if (transpose && b.nchunks > 0) {
      if (f32)
        launch_apply_gemv<float>(b.d_ops, b.d_chunks, b.nchunks, true, x, stage, work, st);
      else
        launch_apply_gemv<double>(b.d_ops, b.d_chunks, b.nchunks, true, x, stage, work, st);
    }
    if (transpose && b.n_nslots > 0)
      launch_apply_nsum(b.d_nslots, b.d_nptr, b.d_noff, b.n_nslots, stage, x, st);
    if (timed) {
      H.kt.close(st);
      H.kt.bytes += b.bytes;
      H.kt.flops += b.flops;
    }
  }
}

void apply_op(Handle& H, bool transpose, double* x, double* stage, double* work, bool timing) {
  apply_op_stream(H, transpose, x, stage, work, timing, H.stream);
}

void apply_op_on(Handle& H, bool transpose, double* x, hipStream_t st) {
  apply_op_stream(H, transpose, x, nullptr, nullptr, false, st);
}

}  // namespace spaqr
