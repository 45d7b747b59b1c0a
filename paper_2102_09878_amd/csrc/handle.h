// The handle behind spaqr_handle: the host plan, device copies of the
// matrix, the factor (device ops + host metadata) and solver workspace.
#pragma once

#include <algorithm>
#include <array>
#include <memory>
#include <string>
#include <vector>

#include "spaqr_impl.h"

struct spaqr_handle_s;

namespace spaqr {

struct OpRec {
  int kind = 0;   // 0 eliminate, 1 scale, 2 sparsify
  int level = 0, round = 0, phase = 0;
  const void* R = nullptr;
  const void* tau = nullptr;
  int64_t ld = 0;
  int n1 = 0, n2 = 0;
  const int* d_s1 = nullptr;
  const int* d_s2 = nullptr;
  std::vector<int> s1, s2;
};

struct ApplyBatch {
  const ApplyOp* d_ops = nullptr;
  int n = 0;
  int max_n1 = 0;
  // W^-T of eliminations: neighbour slots touched by the batch, each with
  // the staging offsets of its contributions in op order (CSR)
  const int* d_nslots = nullptr;
  const int* d_nptr = nullptr;
  const int* d_noff = nullptr;
  int n_nslots = 0;
  // (op, chunk) work-groups of the elimination neighbour products
  const int2* d_chunks = nullptr;
  int nchunks = 0;
  double bytes = 0.0;  // algorithmic bytes of one application of the batch
  double flops = 0.0;
};

// Opt-in per-launch timing of one kernel family.  Families whose kernels
// stamp themselves ("pqr_step") record, per timed launch, the earliest
// work-group start and the latest work-group end read from the GPU's
// constant-rate real-time counter (the kernel's own duration, as a profiler
// reports it); the others are bracketed with HIP events (which also count
// the launch gap).
struct KernelTimer {
  std::string family;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  int64_t calls = 0, seen = 0;
  int every = 1;
  double seconds = 0.0, bytes = 0.0, flops = 0.0;
  // in-kernel spans (first work-group start to last work-group end)
  int64_t span_calls = 0;
  double span_seconds = 0.0;
  // device stamps: STAMP_SLOTS x STAMP_STRIDE words per timed launch
  unsigned long long* d_stamp = nullptr;
  size_t stamp_cap = 0, stamp_used = 0;
  double clock_hz = 0.0;

  bool on(const char* f) const { return !family.empty() && family == f; }
  // true for the launches that are timed (every `every`-th one of the family)
  bool pick(const char* f) { return on(f) && (seen++ % every) == 0; }
  // events come in pairs: mark() opens a timed stretch, close() ends it
  // after the n launches it covered
  std::vector<int> runs;
  void mark(hipStream_t s) {
    if (used == pool.size()) {
      hipEvent_t e;
      SPAQR_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    SPAQR_HIP(hipEventRecord(pool[used++], s));
  }
  void close(hipStream_t s, int n = 1) {
    mark(s);
    runs.push_back(n);
  }

  // Slot for the next timed launch.  Slots start at zero; a kernel folds
  // ~start and end into them with atomicMax, so no per-launch reset is
  // needed (the buffer is cleared when it is created and after a harvest).
  unsigned long long* stamp(hipStream_t s) {
    const size_t per = (size_t)STAMP_SLOTS * STAMP_STRIDE;
    if (stamp_used == stamp_cap) {
      const size_t cap = std::max<size_t>(2048, 2 * stamp_cap);
      unsigned long long* n = nullptr;
      SPAQR_HIP(hipMalloc(&n, cap * per * sizeof(unsigned long long)));
      SPAQR_HIP(hipMemsetAsync(n, 0, cap * per * sizeof(unsigned long long), s));
      if (d_stamp) {
        SPAQR_HIP(hipMemcpyAsync(n, d_stamp, stamp_used * per * sizeof(unsigned long long),
                                 hipMemcpyDeviceToDevice, s));
        SPAQR_HIP(hipStreamSynchronize(s));
        SPAQR_HIP(hipFree(d_stamp));
      }
      d_stamp = n;
      stamp_cap = cap;
      stamp_stream = s;
    }
    return d_stamp + per * stamp_used++;
  }
  hipStream_t stamp_stream = nullptr;
  void harvest_stamps() {
    if (!stamp_used) return;
    if (clock_hz == 0.0) {
      int dev = 0, khz = 0;
      SPAQR_HIP(hipGetDevice(&dev));
      SPAQR_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
      clock_hz = khz * 1e3;
    }
    const size_t per = (size_t)STAMP_SLOTS * STAMP_STRIDE;
    std::vector<unsigned long long> h(per * stamp_used);
    SPAQR_HIP(hipMemcpy(h.data(), d_stamp, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < stamp_used; ++k) {
      unsigned long long t0 = ~0ull, t1 = 0;
      for (int sl = 0; sl < STAMP_SLOTS; ++sl) {
        const unsigned long long* e = h.data() + per * k + (size_t)sl * STAMP_STRIDE;
        if (e[0] == 0) continue;  // no work-group used this slot
        t0 = std::min(t0, ~e[0]);
        t1 = std::max(t1, e[1]);
      }
      if (t0 != ~0ull && t1 >= t0) {
        span_seconds += (double)(t1 - t0) / clock_hz;
        ++span_calls;
      }
    }
    SPAQR_HIP(hipMemsetAsync(d_stamp, 0, h.size() * sizeof(unsigned long long), stamp_stream));
    stamp_used = 0;
  }
  // call after the stream has been synchronised
  void harvest() {
    harvest_stamps();
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      SPAQR_HIP(hipEventElapsedTime(&ms, pool[i], pool[i + 1]));
      seconds += ms * 1e-3;
      calls += i / 2 < runs.size() ? runs[i / 2] : 1;
    }
    used = 0;
    runs.clear();
  }
  void reset(const char* f, int ev) {
    family = f ? f : "";
    every = ev > 0 ? ev : 1;
    used = 0;
    runs.clear();
    if (d_stamp)
      SPAQR_HIP(hipMemset(d_stamp, 0, stamp_cap * STAMP_SLOTS * STAMP_STRIDE * sizeof(unsigned long long)));
    stamp_used = 0;
    calls = 0;
    seen = 0;
    seconds = bytes = flops = 0.0;
    span_calls = 0;
    span_seconds = 0.0;
  }
  ~KernelTimer() {
    for (auto e : pool) (void)hipEventDestroy(e);
    if (d_stamp) (void)hipFree(d_stamp);
  }
};

// Launch shapes chosen per problem by spaqr_autotune (defaults otherwise).
struct TuneParams {
  int pqr_poll = 16;        // pivot steps launched ahead of the last step the GPU has reported
  int pqr_reg_rows = 1024;  // tallest 64-aligned window kept in registers by a pivot step
  int tall_coop = 1;        // tall panels in one cooperative launch (else two launches per column)
};

// Column slots of a group's data: the slots of the clusters it was built
// from, one block after the other, with each block's (cluster, begin, end).
// Immutable once built and shared between groups (and, for the initial
// groups, between factorizations).
struct SlotList {
  std::vector<int> v;
  std::vector<std::array<int, 3>> blk;
};

struct Handle {
  std::string err;
  TuneParams tune;
  spaqr_options opt{};
  Plan P;
  hipStream_t stream = nullptr;
  bool dev_ready = false;
  // device copies of the matrix (scaled values A D^-1 and its transpose)
  double* d_ahat = nullptr;
  int64_t* d_rp = nullptr;
  int32_t* d_ci = nullptr;
  double* d_ahatT = nullptr;
  int64_t* d_atp = nullptr;
  int32_t* d_ati = nullptr;
  int64_t* d_init_dst = nullptr;
  double* d_D = nullptr;
  double* d_vals = nullptr;     // values of A as given (CSR order)
  int64_t* d_atsrc = nullptr;   // CSR entry of each transposed entry
  int* d_flag = nullptr;
  int64_t* d_segc = nullptr;    // problem offsets over columns / rows (count + 1)
  int64_t* d_segr = nullptr;
  int* d_act = nullptr;         // per-problem "still iterating" flags
  int* d_pqr_err = nullptr;     // persistent pivoted QR: set when a wait was abandoned
  std::vector<double> normA;    // ||A_g||_2 estimate of each problem's current values
  size_t plan_bytes = 0;
  // factor
  Arena arena;
  Staging stage;
  bool factored = false;
  int precision = SPAQR_FP64;
  std::vector<OpRec> ops;
  std::vector<ApplyBatch> batches;
  double* d_nstage = nullptr;  // contributions R_sN^T x_s of one batch (arena)
  double* d_awork = nullptr;   // chunk partials / t vectors of one batch (arena)
  int64_t nstage_elems = 0;    // sizes of those two (doubles)
  int64_t awork_elems = 0;
  std::vector<int> ranks;
  spaqr_stats stats{};
  KernelTimer kt;
  // CGLS iteration captured as a HIP graph (recorded on cap_stream, launched
  // on stream).  Its launches depend only on the apply batches' launch
  // arguments (apply_key, a hash of every pointer and size they pass) and
  // on the workspace (cg_base): a refactorization that reproduces both (the
  // same structure allocates the same addresses) keeps the graph.
  uint64_t factor_gen = 0;
  uint64_t apply_key = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t cg_graph = nullptr;
  hipGraphExec_t cg_exec = nullptr;
  uint64_t cg_key = 0;
  const double* cg_base = nullptr;
  void drop_cg_graph();
  // solver workspace
  double* d_cg = nullptr;
  size_t cg_elems = 0;
  double* h_sc = nullptr;  // pinned scalars (count * 8 + 64 doubles)
  int* h_act = nullptr;    // pinned flags (count ints)
  // progress word of the pivot-step loop: written by the step kernels
  // (coherent pinned host memory), read by the host without synchronising
  unsigned long long* h_pqr_report = nullptr;
  unsigned long long* d_pqr_report = nullptr;
  unsigned pqr_tag = 0;
  // slot lists of the initial groups (structural: built by the first
  // factorization, reused by the next ones)
  std::vector<std::shared_ptr<const SlotList>> init_slots;

  ~Handle();
  void ensure_device();
  void release_device();
};

void factorize(Handle& H, double eps, const int* forced, int nforced);
// W^-1 (or W^-T) applied in place to x_dev, batch by batch.  stage / work
// default to the handle's staging buffers (d_nstage, d_awork); timing off
// skips the per-kernel timer (which may allocate event and stamp storage).
void apply_op(Handle& H, bool transpose, double* x_dev, double* stage = nullptr, double* work = nullptr,
              bool timing = true);
// The same on stream st, with the handle's staging and no timing (for
// recording into a graph).
void apply_op_on(Handle& H, bool transpose, double* x_dev, hipStream_t st);
// CGLS on every problem of the plan at once, each with its own scalars and
// stopping test; infos[count] (may be null).  Returns SPAQR_NOCONV if any
// problem reached max_iter.
int cgls(Handle& H, const double* b, double tol, int max_iter, double* x, spaqr_cgls_info* infos);
void csne(Handle& H, const double* b, double* x);
// Corrected seminormal equations with iterative refinement (Section 1);
// infos[count] (may be null).  SPAQR_NOCONV if a problem missed tol.
int csne_refine(Handle& H, const double* b, double tol, int max_steps, double* x, spaqr_cgls_info* infos);
// The same solve with every intermediate in the library's static device
// scratch array (no device allocation in the call).
void csne_noalloc(Handle& H, const double* b, double* x);
// Column scaling of the current device values d_vals: D, Ahat, Ahat^T and
// the ||A||_2 estimate, all on the device.
void scale_values(Handle& H);
void check_tune(const TuneParams& t);
void autotune(Handle& H, double eps, int reps, const char* cache_path, spaqr_tune* out);
int adjoint(Handle& H, const double* x, const double* b, const double* g, double tol, int max_iter,
            double* grad_b, double* grad_vals, double* lambda, spaqr_cgls_info* info);

}  // namespace spaqr
