// Batched column-pivoted Householder QR for gfx950, one launch per pivot
// step.  Used for the rank-revealing QRs of the paper: the rows below the
// diagonal of an eliminated cluster (Section 4.2), the rows below an
// interface's scaled diagonal (step 1, Section 2.5.1) and [A_np^T A_p1n]
// (step 2, Section 2.5.2).
//
// The matrices are short and wide or just large (e.g. 126 x 11000,
// 630 x 3000), and one pivot step touches every remaining column.  Each
// matrix is therefore split into chunks of PQR_CW columns, one work-group
// per chunk; a work-group owns its columns' data and FP64 norms.  The kernel
// boundary between steps is the only synchronisation: step i reads the
// per-chunk argmax written by step i-1, every work-group recomputes the same
// reflector from the pivot column, applies it to its own columns, downdates
// their norms (LAPACK Working Note 176 rule) and publishes its next argmax.
// The pivot column itself is finalised (beta on the diagonal, zeros below)
// one step later, after every work-group has read it.
//
// Rank rule (Section 4): stop at the first step whose |R_ii| is below
// eps |R_00| (unless the matrix is marked exact), or at or below the
// numerical-rank floor noise * ||A||_F, or when `forced` steps were taken.  Pivot ties go to the lowest column index.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cstdlib>

#include "spaqr_impl.h"
#include "wave.h"

namespace spaqr {

namespace {

constexpr int BS = 256;
constexpr int PL = 6;  // chunk partials per thread fetched up front
static_assert(PQR_CW == 8, "a pivot step gives each of its 4 waves cw/4 columns");

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum63(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// block-wide argmax of (val, idx): larger val wins, lowest idx on ties
__device__ __forceinline__ void block_argmax(double& bv, int& bi, double* shv, int* shi) {
  wave_argmax_dpp(bv, bi);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) shv[threadIdx.x >> 6] = bv, shi[threadIdx.x >> 6] = bi;
  __syncthreads();
  bv = shv[0];
  bi = shi[0];
  for (int w = 1; w < 4; ++w)
    if (shv[w] > bv || (shv[w] == bv && shi[w] < bi)) bv = shv[w], bi = shi[w];
}

// Reflector scalars in LAPACK's convention (beta = -sign(alpha) ||x||,
// sign(0) = +1), where an alpha of at most SIGN_FLOOR u ||x|| (u the FP64
// unit roundoff, whatever the storage type) counts as 0: it is a structural
// zero carrying rounding error, whose sign two evaluations may not agree
// on.  (FP32 rounding can exceed that floor; there the FP32 form may flip
// an R row relative to the FP64 form: an equivalent factor.)
constexpr double SIGN_FLOOR = 64.0 * 1.1102230246251565e-16;
__device__ __forceinline__ void house_scalars(double alpha, double xn2, double& beta, double& tau,
                                              double& scal) {
  if (xn2 == 0.0) {
    beta = alpha;
    tau = 0.0;
    scal = 1.0;
  } else {
    const double nrm = sqrt(alpha * alpha + xn2);
    const double s = (alpha < 0.0 && -alpha > SIGN_FLOOR * nrm) ? -1.0 : 1.0;
    beta = -s * nrm;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
}

// Local argmax over the chunk's live columns (done == 0, not `skip`).
__device__ __forceinline__ void chunk_argmax(const double* vn1, const double* done, int c0, int c1,
                                             int skip, double& bv, int& bi, double* shv, int* shi) {
  bv = -1.0;
  bi = INT_MAX;
  for (int j = c0 + (int)threadIdx.x; j < c1; j += BS)
    if (j != skip && done[j] == 0.0 && vn1[j] > bv) bv = vn1[j], bi = j;
  block_argmax(bv, bi, shv, shi);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_pqr_init(const PQRDesc* __restrict__ D,
                                                 PQRState* __restrict__ S, PQRPart* __restrict__ parts,
                                                 double* __restrict__ frop, const int2* __restrict__ bmap) {
  const int2 bm = bmap[blockIdx.x];
  const PQRDesc d = D[bm.x];
  const T* A = static_cast<const T*>(d.A);
  double* vn1 = d.work;
  double* vn2 = d.work + d.n;
  double* done = d.work + 2 * d.n;
  const int c0 = bm.y * d.cw, c1 = min(d.n, c0 + d.cw);
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  __shared__ double sh[4];
  __shared__ double shv[4];
  __shared__ int shi[4];
  double fro = 0.0;
  for (int j = c0 + wv; j < c1; j += 4) {
    const T* y = A + (int64_t)j * d.lda;
    double s = 0.0;
    for (int r = lane; r < d.m; r += 64) s += (double)y[r] * (double)y[r];
    s = wave_sum(s);
    if (lane == 0) {
      fro += s;
      vn1[j] = sqrt(s);
      vn2[j] = sqrt(s);
      done[j] = 0.0;
    }
  }
  fro = block_sum(fro, sh);
  double bv;
  int bi;
  chunk_argmax(vn1, done, c0, c1, -1, bv, bi, shv, shi);
  if (tid == 0) {
    PQRPart p;
    p.val = bv;
    p.idx = bi;
    p.pad_ = 0;
    parts[d.blk0 + bm.y] = p;
    frop[d.blk0 + bm.y] = fro;
    if (bm.y == 0) {
      PQRState s;
      s.r00 = 0.0;
      s.floor = 0.0;
      s.beta = 0.0;
      s.pivot = -1;
      s.pstep = -1;
      s.rank = 0;
      s.stopped = min(d.m, d.n) == 0 ? 1 : 0;
      S[2 * bm.x] = s;
    }
  }
}

// PQ: rows per lane held in registers for this work-group's columns (the
// launcher picks 2 to 16 when that covers the batch's tallest matrix from
// the step's 64-aligned row window; 0 keeps the columns in memory).
// NC = cw / 4 columns per wave.
// Optional self-timing: when stamp is set, thread 0 of every work-group
// folds the complement of the real-time counter into its slot's first word
// on entry (so the maximum is the earliest start) and the counter into the
// second word on exit.  Work-groups spread over STAMP_SLOTS slots, one
// 64-byte line apart, to keep the atomics from queueing on one address.
struct StampScope {
  unsigned long long* p;
  __device__ explicit StampScope(unsigned long long* q)
      : p(q ? q + (blockIdx.x % STAMP_SLOTS) * STAMP_STRIDE : nullptr) {
    if (p && threadIdx.x == 0) atomicMax(p, ~(unsigned long long)__builtin_amdgcn_s_memrealtime());
  }
  __device__ ~StampScope() {
    if (p && threadIdx.x == 0) atomicMax(p + 1, (unsigned long long)__builtin_amdgcn_s_memrealtime());
  }
};

// CF: the work-group reads its matrix's state before fetching anything else
// and does nothing more once that matrix has stopped (batches of many
// matrices, whose ranks differ); without it every fetch is issued at once
// (one round trip less per step, for the chains of single matrices).
template <typename T, int PQ, int NC, bool CF>
__global__ __launch_bounds__(BS) void k_pqr_step(const PQRDesc* __restrict__ D, PQRState* __restrict__ S,
                                                 PQRPart* __restrict__ parts, int total_parts,
                                                 const double* __restrict__ frop,
                                                 const int2* __restrict__ bmap, int* __restrict__ active,
                                                 int i, double eps, unsigned long long* stamp,
                                                 unsigned long long* report, unsigned tag) {
  const StampScope timing(stamp);
  // progress for the host, which then needs no stream synchronisation to
  // stop launching steps: the matrices still running after step i - 1
  // (final at this kernel's start), tagged with the batch and the step
  if (report && blockIdx.x == 0 && threadIdx.x == 0) {
    const int a = __hip_atomic_load(active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long w = ((unsigned long long)(tag & 0xFFFFFFu) << 40) |
                                 ((unsigned long long)(unsigned)i << 20) | (unsigned)min(max(a, 0), 0xFFFFF);
    __hip_atomic_store(report, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  extern __shared__ double x[];  // pivot column rows i..m-1
  __shared__ double sh[4];
  __shared__ double shv[4];
  __shared__ int shi[4];
  // Loads are issued in the order they are needed (they complete in
  // order): block map with this work-group's own copy of its matrix's
  // descriptor (no second round trip to find it), state and chunk
  // partials, then the work-group's own columns, which are consumed last.
  const int2 bm = bmap[blockIdx.x];
  const PQRDesc d = D[blockIdx.x];
  const int mi = bm.x, ch = bm.y;
  const PQRState sp = S[2 * mi + (i & 1)];
  PQRState* sn = S + 2 * mi + ((i + 1) & 1);
  const PQRPart* prd = parts + (size_t)(i & 1) * total_parts;
  PQRPart* pwr = parts + (size_t)((i + 1) & 1) * total_parts;
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int m = d.m, n = d.n;
  const int c0 = ch * d.cw, c1 = min(n, c0 + d.cw);
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  double* vn1 = d.work;
  double* vn2 = d.work + n;
  double* done = d.work + 2 * n;
  const bool idle = CF && sp.stopped;
  double pval[PL];
  int pidx[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int k = tid + u * BS;
    if (!idle && k < d.nblk) {
      const PQRPart q = prd[d.blk0 + k];
      pval[u] = q.val, pidx[u] = q.idx;
    } else {
      pval[u] = -1.0, pidx[u] = INT_MAX;
    }
  }
  // squared Frobenius norm (first step only): thread t sums chunks t, t + BS, ...
  double fro = 0.0;
  if (i == 0 && !idle)
    for (int k = tid; k < d.nblk; k += BS) fro += frop[d.blk0 + k];
  // Register rows form a 64-aligned window: lane l holds rows i0 + l + 64 q,
  // so every per-lane partial sum runs over the rows congruent to l mod 64
  // in ascending order, whatever the step (the persistent form below keeps
  // the same grouping and gives bit-identical factors).
  const int i0 = i & ~63;
  const bool regs = PQ > 0 && m - i0 <= 64 * PQ;
  int jcol[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) jcol[k] = c0 + wv + 4 * k;
  T yv[NC][PQ > 0 ? PQ : 1];  // values of the storage type (exactly what memory holds)
  double v1p[NC], v2p[NC], dnp[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) v1p[k] = 0.0, v2p[k] = 1.0, dnp[k] = 1.0;
  if (regs && !idle) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int j = jcol[k] < c1 ? jcol[k] : c0;
      const T* y = A + (int64_t)j * lda;
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int r = i0 + lane + 64 * q;
        yv[k][q] = (r >= i && r < m) ? y[r] : T(0);
      }
      dnp[k] = done[j];
      v1p[k] = vn1[j];
      v2p[k] = vn2[j];
    }
  }

  // finalise the previous pivot column (idempotent; every reader is done with it)
  if (sp.pivot >= c0 && sp.pivot < c1) {
    T* col = A + (int64_t)sp.pivot * lda;
    if (tid == 0) col[sp.pstep] = static_cast<T>(sp.beta);
    for (int r = sp.pstep + 1 + tid; r < m; r += BS) col[r] = T(0);
  }
  if (sp.stopped) {
    if (ch == 0 && tid == 0) *sn = sp;
    return;
  }
  // global pivot and (first step) the Frobenius norm
  double bv = -1.0;
  int bi = INT_MAX;
#pragma unroll
  for (int u = 0; u < PL; ++u)
    if (pval[u] > bv || (pval[u] == bv && pidx[u] < bi)) bv = pval[u], bi = pidx[u];
  for (int k = tid + PL * BS; k < d.nblk; k += BS) {
    const PQRPart q = prd[d.blk0 + k];
    if (q.val > bv || (q.val == bv && q.idx < bi)) bv = q.val, bi = q.idx;
  }
  block_argmax(bv, bi, shv, shi);
  double floor_v = sp.floor;
  if (i == 0) floor_v = d.noise * sqrt(block_sum(fro, sh));
  const int p = bi;
  bool stop = i >= min(m, n) || p < 0 || p >= n || bv < 0.0;
  double beta = 0.0, tv = 0.0, scal = 1.0, r00 = sp.r00;
  if (!stop) {
    const T* col = A + (int64_t)p * lda;
    double part = 0.0;
    for (int r = i + tid; r < m; r += BS) {
      const double v = col[r];
      x[r - i] = v;
      if (r > i) part += v * v;
    }
    const double xn2 = block_sum(part, sh);
    const double alpha = x[0];
    house_scalars(alpha, xn2, beta, tv, scal);
    if (i == 0) r00 = fabs(beta);
    stop = fabs(beta) <= floor_v;
    if (d.forced >= 0)
      stop = stop || i >= d.forced;
    else if (i > 0 && !d.exact)
      stop = stop || fabs(beta) < eps * r00;
  }
  if (stop) {
    if (ch == 0 && tid == 0) {
      PQRState s = sp;
      s.stopped = 1;
      s.floor = floor_v;
      s.r00 = r00;
      *sn = s;
      atomicSub(active, 1);
    }
    return;
  }
  // reflector v (v[0] = 1) in LDS
  if (tv != 0.0)
    for (int r = 1 + tid; r < m - i; r += BS) x[r] *= scal;
  __syncthreads();
  if (tid == 0) x[0] = 1.0;
  __syncthreads();
  if (ch == 0) {
    if (d.V) {
      T* vc = static_cast<T*>(d.V) + (int64_t)i * m;
      for (int r = tid; r < m; r += BS) vc[r] = r < i ? T(0) : static_cast<T>(x[r - i]);
    }
    if (tid == 0) {
      if (d.tau) static_cast<T*>(d.tau)[i] = static_cast<T>(tv);
      if (d.piv_out) d.piv_out[i] = p;
      PQRState s;
      s.r00 = r00;
      s.floor = floor_v;
      s.beta = beta;
      s.pivot = p;
      s.pstep = i;
      s.rank = i + 1;
      s.stopped = 0;
      *sn = s;
    }
  }
  // apply H_i to the chunk's live columns and downdate their norms
  const double tol3z = sqrt(DBL_EPSILON);
  // register path: the wave's best live column after the update (its norms
  // are wave-uniform), so the chunk argmax needs no second read of them
  double cv = -1.0;
  int ci = INT_MAX;
  if (regs) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int j = jcol[k];
      if (j >= c1 || j == p || dnp[k] != 0.0) continue;
      T* y = A + (int64_t)j * lda;
      double dot = 0.0;
      if (tv != 0.0)
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int r = i0 + lane + 64 * q;
          if (r >= i && r < m) dot += x[r - i] * (double)yv[k][q];
        }
      dot = wave_sum(dot);
      const double f = tv * dot;
      const double yi = (double)lane_bcast(yv[k][0], i - i0) - f;
      if (tv != 0.0)
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int r = i0 + lane + 64 * q;
          if (r >= i && r < m) {
            const T nv = static_cast<T>((double)yv[k][q] - f * x[r - i]);
            y[r] = nv;
            yv[k][q] = nv;
          }
        }
      const double v1 = v1p[k];
      double nv1 = v1;
      if (v1 != 0.0) {
        const double ay = fabs((double)static_cast<T>(yi));
        double temp = 1.0 - (ay / v1) * (ay / v1);
        temp = temp > 0.0 ? temp : 0.0;
        const double ratio = v1 / v2p[k];
        const double temp2 = temp * ratio * ratio;
        if (temp2 <= tol3z) {
          double s2 = 0.0;
#pragma unroll
          for (int q = 0; q < PQ; ++q) {
            const int r = i0 + lane + 64 * q;
            if (r > i && r < m) s2 += (double)yv[k][q] * (double)yv[k][q];
          }
          s2 = sqrt(wave_sum(s2));
          nv1 = s2;
          if (lane == 0) vn1[j] = s2, vn2[j] = s2;
        } else {
          nv1 = v1 * sqrt(temp);
          if (lane == 0) vn1[j] = nv1;
        }
      }
      // ascending columns: the first of equal norms wins, as in chunk_argmax
      if (nv1 > cv) cv = nv1, ci = j;
    }
  }
  for (int j = c0 + wv; !regs && j < c1; j += 4) {
    if (j == p || done[j] != 0.0) continue;
    T* y = A + (int64_t)j * lda;
    double dot = 0.0;
    const int rl = i0 + lane < i ? i0 + lane + 64 : i0 + lane;  // first row >= i congruent to lane
    if (tv != 0.0)
      for (int r = rl; r < m; r += 64) dot += x[r - i] * (double)y[r];
    dot = wave_sum(dot);
    const double f = tv * dot;
    const double yi = (double)y[i] - f;
    if (tv != 0.0)
      for (int r = rl; r < m; r += 64) y[r] = static_cast<T>((double)y[r] - f * x[r - i]);
    const double v1 = vn1[j];
    if (v1 != 0.0) {
      const double ay = fabs((double)static_cast<T>(yi));
      double temp = 1.0 - (ay / v1) * (ay / v1);
      temp = temp > 0.0 ? temp : 0.0;
      const double ratio = v1 / vn2[j];
      const double temp2 = temp * ratio * ratio;
      if (temp2 <= tol3z) {
        double s = 0.0;
        for (int r = rl + (rl == i ? 64 : 0); r < m; r += 64) s += (double)y[r] * (double)y[r];
        s = sqrt(wave_sum(s));
        if (lane == 0) vn1[j] = s, vn2[j] = s;
      } else if (lane == 0) {
        vn1[j] = v1 * sqrt(temp);
      }
    }
  }
  if (tid == 0 && p >= c0 && p < c1) done[p] = 1.0;
  if (regs) {
    // every wave has passed the barriers after the pivot argmax's reads of
    // shv / shi, so they can be reused here
    if (lane == 0) shv[wv] = cv, shi[wv] = ci;
    __syncthreads();
    bv = shv[0];
    bi = shi[0];
    for (int w = 1; w < 4; ++w)
      if (shv[w] > bv || (shv[w] == bv && shi[w] < bi)) bv = shv[w], bi = shi[w];
  } else {
    __syncthreads();
    chunk_argmax(vn1, done, c0, c1, p, bv, bi, shv, shi);
  }
  if (tid == 0) {
    PQRPart q;
    q.val = bv;
    q.idx = bi;
    q.pad_ = 0;
    pwr[d.blk0 + ch] = q;
  }
}

// ---------------------------------------------------------------------------
// Persistent form: one cooperative launch runs every pivot step of a batch.
//
// Each work-group is one wave and owns a chunk of NCW columns of one matrix,
// held in registers for the whole factorization (lane l holds rows l + 64 q,
// the grouping of the per-step kernel, so every sum is formed in the same
// order and the factors are bit-identical); lane k keeps column k's norms.
// Waves exchange data only through 64-bit words whose low half carries the
// number of the step the data is for (values are split into 32-bit halves):
// at the end of a step a wave writes its chunk argmax and that candidate
// column for the next step, and a step starts once the reader has seen the
// current tag on every chunk argmax of its matrix; the pivot column is then
// read from its owner's candidate words the same way.  No flags, fences or
// barriers are needed: a word is either old (wrong tag) or complete.  Two
// slots alternate by step parity; a slot is rewritten two steps later, after
// every wave of the matrix has published the step in between and so has
// finished reading it.  The buffers are zeroed before the launch (tag 0 is
// never current).  Matrices never wait on each other, and all waves of a
// matrix reach the same stop decision at the same step.  Every wait is
// bounded: past 100 ms a wave raises `err` and exits, and the others exit
// when they see it.
// ---------------------------------------------------------------------------
constexpr unsigned long long PQR_WAIT_TICKS = 10000000ull;  // 100 ms at 100 MHz
constexpr int PQR_RUN_MAX_WAVES = 1000;
constexpr int PQR_POLL = 8;  // chunk argmax words per lane and poll: matrices up to 512 chunks

typedef unsigned long long u64;

__device__ __forceinline__ void st_tag(u64* p, unsigned hi, unsigned tag) {
  __hip_atomic_store(p, ((u64)hi << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 ld_tag(const u64* p) {
  return __hip_atomic_load(const_cast<u64*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool tag_ok(u64 w, unsigned tag) { return (unsigned)w == tag; }
__device__ __forceinline__ unsigned hi_of(u64 w) { return (unsigned)(w >> 32); }

template <typename T>
struct Tagged;
template <>
struct Tagged<float> {
  static constexpr int W = 1;  // 64-bit words per value
  __device__ static void put(u64* p, float v, unsigned tag) { st_tag(p, __float_as_uint(v), tag); }
  __device__ static bool get(const u64* p, unsigned tag, float& v) {
    const u64 a = ld_tag(p);
    v = __uint_as_float(hi_of(a));
    return tag_ok(a, tag);
  }
};
template <>
struct Tagged<double> {
  static constexpr int W = 2;
  __device__ static void put(u64* p, double v, unsigned tag) {
    const u64 b = (u64)__double_as_longlong(v);
    st_tag(p, (unsigned)(b >> 32), tag);
    st_tag(p + 1, (unsigned)b, tag);
  }
  __device__ static bool get(const u64* p, unsigned tag, double& v) {
    const u64 a = ld_tag(p), b = ld_tag(p + 1);
    v = __longlong_as_double((long long)(((u64)hi_of(a) << 32) | hi_of(b)));
    return tag_ok(a, tag) && tag_ok(b, tag);
  }
};

__device__ __forceinline__ bool wave_all(bool ok) { return __ballot(!ok) == 0; }

// Bookkeeping of one wait, bounded by elapsed time on the constant-rate
// real-time counter (100 MHz): false once the wait is abandoned, after
// PQR_WAIT_TICKS or as soon as another wave has raised `err`.
struct WaitClock {
  unsigned long long t0 = 0;
  unsigned polls = 0;
};
__device__ __forceinline__ bool keep_waiting(WaitClock& w, int* err) {
  const unsigned long long now = __builtin_amdgcn_s_memrealtime();
  if (w.polls++ == 0) w.t0 = now;
  if (now - w.t0 > PQR_WAIT_TICKS) {
    atomicOr(err, 1);
    return false;
  }
  if ((w.polls & 31) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
  __builtin_amdgcn_s_sleep(1);
  return true;
}

// wave argmax of (val, idx): larger val wins, lowest idx on ties
__device__ __forceinline__ void wave_argmax(double& bv, int& bi) { wave_argmax_dpp(bv, bi); }

template <typename T, int PQ, int NCW>
__global__ __launch_bounds__(64) void k_pqr_run(const PQRDesc* __restrict__ D, const int2* __restrict__ bmap,
                                                PQRXch xc, double eps, unsigned long long* stamp) {
  typedef Tagged<T> TG;
  const StampScope timing(stamp);
  const int2 bm = bmap[blockIdx.x];
  const PQRDesc d = D[bm.x];
  const int ch = bm.y;
  const int m = d.m, n = d.n;
  const int c0 = ch * NCW, c1 = min(n, c0 + NCW);
  const int gb = d.blk0 + ch;
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int lane = threadIdx.x;
  const double tol3z = sqrt(DBL_EPSILON);
  const size_t pub_stride = (size_t)xc.rows * TG::W;
  // a valid rank even if a wait is abandoned (the caller then reports the error)
  if (ch == 0 && lane == 0) d.rank_out[0] = 0;

  // columns c0 .. c0 + NCW - 1 into registers; lane k keeps column k's norms
  T y[NCW][PQ];
  double s[NCW];
#pragma unroll
  for (int k = 0; k < NCW; ++k) {
    const int j = c0 + k;
    const T* col = A + (int64_t)(j < c1 ? j : 0) * lda;
    s[k] = 0.0;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int r = lane + 64 * q;
      y[k][q] = (j < c1 && r < m) ? col[r] : T(0);
      if (r < m) s[k] += (double)y[k][q] * (double)y[k][q];
    }
  }
#pragma unroll
  for (int k = 0; k < NCW; ++k) s[k] = wave_sum(s[k]);
  double myv1 = 0.0;
#pragma unroll
  for (int k = 0; k < NCW; ++k)
    if (lane == k) myv1 = sqrt(s[k]);
  double myv2 = myv1;
  bool mydone = !(lane < NCW && c0 + lane < c1);
  // squared Frobenius norm per 8-column group, summed as the per-step
  // initialisation does (its 4 waves take columns v and v + 4 of the group)
#pragma unroll
  for (int g = 0; g < NCW / 8; ++g) {
    double w[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 8 * g + v, b = a + 4;
      w[v] = c0 + a < c1 ? s[a] : 0.0;
      if (c0 + b < c1) w[v] += s[b];
    }
    if (lane == g && c0 + 8 * g < n) {
      u64* f = xc.frop + 2 * ((size_t)d.g0 + ch * (NCW / 8) + g);
      Tagged<double>::put(f, (w[0] + w[1]) + (w[2] + w[3]), 1u);
    }
  }

  // publishes the chunk argmax and its candidate column (rows `from` and
  // below) for the step whose tag is `tag`, into slot `slot`
  auto publish = [&](int slot, unsigned tag, int from) {
    double bv = (!mydone) ? myv1 : -1.0;
    int bi = (!mydone) ? c0 + lane : INT_MAX;
    wave_argmax(bv, bi);
    if (bi != INT_MAX) {
      const int ks = bi - c0;
      u64* pub = xc.pub + ((size_t)slot * xc.G + gb) * pub_stride;
#pragma unroll
      for (int k = 0; k < NCW; ++k)
        if (k == ks)
#pragma unroll
          for (int q = 0; q < PQ; ++q) {
            const int r = lane + 64 * q;
            if (r >= from && r < m) TG::put(pub + (size_t)r * TG::W, y[k][q], tag);
          }
    }
    if (lane == 0) {
      u64* pw = xc.part + 3 * ((size_t)slot * xc.G + gb);
      const u64 b = (u64)__double_as_longlong(bv);
      st_tag(pw, (unsigned)(b >> 32), tag);
      st_tag(pw + 1, (unsigned)b, tag);
      st_tag(pw + 2, (unsigned)bi, tag);
    }
  };
  publish(0, 1u, 0);

  double r00 = 0.0, floor_v = 0.0;
  const int kmax = min(m, n);
  int i = 0;
  for (;; ++i) {
    const unsigned tag = (unsigned)i + 1u;
    const int slot = i & 1;
    // global argmax over the chunk candidates of this matrix
    double bv = -1.0;
    int bi = INT_MAX;
    {
      const u64* pr = xc.part + 3 * ((size_t)slot * xc.G + d.blk0);
      WaitClock spins;
      for (;;) {
        bool ok = true;
        double lv = -1.0;
        int li = INT_MAX;
        u64 w0[PQR_POLL], w1[PQR_POLL], w2[PQR_POLL];
#pragma unroll
        for (int u = 0; u < PQR_POLL; ++u) {
          const int k = lane + 64 * u;
          if (k < d.nblk) {
            w0[u] = ld_tag(pr + 3 * k);
            w1[u] = ld_tag(pr + 3 * k + 1);
            w2[u] = ld_tag(pr + 3 * k + 2);
          }
        }
#pragma unroll
        for (int u = 0; u < PQR_POLL; ++u) {
          const int k = lane + 64 * u;
          if (k < d.nblk) {
            ok = ok && tag_ok(w0[u], tag) && tag_ok(w1[u], tag) && tag_ok(w2[u], tag);
            const double v = __longlong_as_double((long long)(((u64)hi_of(w0[u]) << 32) | hi_of(w1[u])));
            const int ix = (int)hi_of(w2[u]);
            if (v > lv || (v == lv && ix < li)) lv = v, li = ix;
          }
        }
        if (wave_all(ok)) {
          bv = lv;
          bi = li;
          break;
        }
        if (!keep_waiting(spins, xc.err)) return;
      }
    }
    wave_argmax(bv, bi);
    const int p = bi;
    bool stop = i >= kmax || p < 0 || p >= n || bv < 0.0;
    // (an empty matrix publishes no Frobenius-norm groups; it stops here)
    if (i == 0 && !stop) {
      // the per-step form's reduction: thread t of 256 sums groups t, t + 256, ...
      const int ng = max(1, (n + 7) / 8);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int gb0 = 0; gb0 < ng; gb0 += 256) {
        double f[4];
        WaitClock spins;
        for (;;) {
          bool ok = true;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int g = gb0 + 64 * v + lane;
            f[v] = 0.0;
            if (g < ng) ok = Tagged<double>::get(xc.frop + 2 * ((size_t)d.g0 + g), 1u, f[v]) && ok;
          }
          if (wave_all(ok)) break;
          if (!keep_waiting(spins, xc.err)) return;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (gb0 + 64 * v + lane < ng) acc[v] += f[v];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = wave_sum(acc[v]);
      floor_v = d.noise * sqrt((acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
    double beta = 0.0, tv = 0.0, scal = 1.0;
    double xr[PQ];  // pivot column, then the reflector, at rows lane + 64 q (zero above row i)
    if (!stop) {
      const u64* pc = xc.pub + ((size_t)slot * xc.G + d.blk0 + p / NCW) * pub_stride;
      double xs[PQ];  // rows i + 64 w + lane, the per-step form's grouping of ||x||^2
      WaitClock spins;
      for (;;) {
        bool ok = true;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int r = lane + 64 * q;
          T v = T(0);
          if (r >= i && r < m) ok = TG::get(pc + (size_t)r * TG::W, tag, v) && ok;
          xr[q] = (double)v;
          const int rs = i + 64 * q + lane;
          T u = T(0);
          if (rs < m) ok = TG::get(pc + (size_t)rs * TG::W, tag, u) && ok;
          xs[q] = (double)u;
        }
        if (wave_all(ok)) break;
        if (!keep_waiting(spins, xc.err)) return;
      }
      double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < PQ && q < 4; ++q) {
        const int rs = i + 64 * q + lane;
        if (rs > i && rs < m) part[q] = xs[q] * xs[q];
      }
#pragma unroll
      for (int w = 0; w < 4; ++w) part[w] = wave_sum(part[w]);
      const double xn2 = (part[0] + part[1]) + (part[2] + part[3]);
      const double alpha = lane_bcast(xs[0], 0);
      house_scalars(alpha, xn2, beta, tv, scal);
      if (i == 0) r00 = fabs(beta);
      stop = fabs(beta) <= floor_v;
      if (d.forced >= 0)
        stop = stop || i >= d.forced;
      else if (i > 0 && !d.exact)
        stop = stop || fabs(beta) < eps * r00;
    }
    if (stop) break;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int r = lane + 64 * q;
      if (r == i)
        xr[q] = 1.0;
      else if (r > i && tv != 0.0)
        xr[q] *= scal;
    }
    if (ch == 0) {
      if (d.V) {
        T* vc = static_cast<T*>(d.V) + (int64_t)i * m;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int r = lane + 64 * q;
          if (r < m) vc[r] = r < i ? T(0) : static_cast<T>(xr[q]);
        }
      }
      if (lane == 0) {
        if (d.tau) static_cast<T*>(d.tau)[i] = static_cast<T>(tv);
        if (d.piv_out) d.piv_out[i] = p;
      }
    }
    // the pivot column goes out final (R entries above, beta, zeros below)
    if (p >= c0 && p < c1) {
#pragma unroll
      for (int k = 0; k < NCW; ++k)
        if (c0 + k == p) {
          T* col = A + (int64_t)p * lda;
#pragma unroll
          for (int q = 0; q < PQ; ++q) {
            const int r = lane + 64 * q;
            if (r < m) col[r] = r < i ? y[k][q] : (r == i ? static_cast<T>(beta) : T(0));
          }
        }
      if (lane == p - c0) mydone = true;
    }
    // H_i on the live columns, all NCW side by side
    const bool mylive = !mydone;
    const unsigned long long livem = __ballot(mylive);
    double dot[NCW];
    T yold[NCW];
#pragma unroll
    for (int k = 0; k < NCW; ++k) {
      dot[k] = 0.0;
      yold[k] = T(0);
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int r = lane + 64 * q;
        if (tv != 0.0 && r >= i && r < m) dot[k] += xr[q] * (double)y[k][q];
        if (q == (i >> 6)) yold[k] = y[k][q];
      }
    }
#pragma unroll
    for (int k = 0; k < NCW; ++k) dot[k] = wave_sum(dot[k]);
    double mydot = 0.0;
    T myyold = T(0);
#pragma unroll
    for (int k = 0; k < NCW; ++k) {
      const T yk = lane_bcast(yold[k], i & 63);
      if (lane == k) mydot = dot[k], myyold = yk;
    }
    if (tv != 0.0)
#pragma unroll
      for (int k = 0; k < NCW; ++k) {
        if (!((livem >> k) & 1)) continue;
        const double f = tv * dot[k];
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int r = lane + 64 * q;
          if (r >= i && r < m) y[k][q] = static_cast<T>((double)y[k][q] - f * xr[q]);
        }
      }
    // norm downdate (LAPACK Working Note 176), lane k for column k
    bool myneed = false;
    double v1n = myv1;
    if (mylive && myv1 != 0.0) {
      const double f = tv * mydot;
      const double yi = (double)myyold - f;
      const double ay = fabs((double)static_cast<T>(yi));
      double temp = 1.0 - (ay / myv1) * (ay / myv1);
      temp = temp > 0.0 ? temp : 0.0;
      const double ratio = myv1 / myv2;
      const double temp2 = temp * ratio * ratio;
      myneed = temp2 <= tol3z;
      v1n = myv1 * sqrt(temp);
    }
    const unsigned long long needm = __ballot(myneed);
    if (needm) {
#pragma unroll
      for (int k = 0; k < NCW; ++k) {
        dot[k] = 0.0;
        if ((needm >> k) & 1)
#pragma unroll
          for (int q = 0; q < PQ; ++q) {
            const int r = lane + 64 * q;
            if (r > i && r < m) dot[k] += (double)y[k][q] * (double)y[k][q];
          }
      }
#pragma unroll
      for (int k = 0; k < NCW; ++k)
        if ((needm >> k) & 1) dot[k] = wave_sum(dot[k]);
#pragma unroll
      for (int k = 0; k < NCW; ++k)
        if (lane == k && myneed) v1n = sqrt(dot[k]);
    }
    if (mylive) {
      myv1 = v1n;
      if (myneed) myv2 = v1n;
    }
    publish(slot ^ 1, tag + 1u, i + 1);
  }
  // stopped at step i: the columns still held go back to A, and the rank out
  const unsigned long long keep = __ballot(!mydone);
#pragma unroll
  for (int k = 0; k < NCW; ++k) {
    if (!((keep >> k) & 1)) continue;
    T* col = A + (int64_t)(c0 + k) * lda;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int r = lane + 64 * q;
      if (r < m) col[r] = y[k][q];
    }
  }
  if (ch == 0 && lane == 0) d.rank_out[0] = i;
}

template <typename T>
__global__ __launch_bounds__(BS) void k_pqr_finish(const PQRDesc* __restrict__ D,
                                                   const PQRState* __restrict__ S, int steps) {
  const PQRDesc d = D[blockIdx.x];
  const PQRState s = S[2 * blockIdx.x + (steps & 1)];
  if (s.pivot >= 0) {
    T* col = static_cast<T*>(d.A) + (int64_t)s.pivot * d.lda;
    if (threadIdx.x == 0) col[s.pstep] = static_cast<T>(s.beta);
    for (int r = s.pstep + 1 + threadIdx.x; r < d.m; r += BS) col[r] = T(0);
  }
  if (threadIdx.x == 0) d.rank_out[0] = s.rank;
}

}  // namespace

template <typename T>
void launch_pqr_init(const PQRDesc* d_desc, int nblocks, PQRState* states, PQRPart* parts, double* frop,
                     const int2* bmap, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_pqr_init<T>, dim3(nblocks), dim3(BS), 0, s, d_desc, states, parts, frop, bmap);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_pqr_step(const PQRDesc* d_blk, int nblocks, int total_parts, PQRState* states,
                     PQRPart* parts, const double* frop, const int2* bmap, int* active, int i, double eps,
                     int max_m, int cw, int reg_rows, unsigned long long* stamp, unsigned long long* report,
                     unsigned tag, bool check_first, hipStream_t s) {
  if (nblocks <= 0) return;
  if (i >= (1 << 20)) throw Error(SPAQR_EARG, "internal: pivot step index beyond the progress word");
  const size_t lds = (size_t)std::max(1, max_m) * sizeof(double);
  if (lds > 64 * 1024) throw Error(SPAQR_EARG, "rank-revealing QR block taller than 8192 rows");
  const int rows = max_m - (i & ~63);
  const bool regs = rows <= std::min(reg_rows, 1024);
#define SPAQR_PQR_GO(Q, C)                                                                                    \
  do {                                                                                                          \
    if (check_first)                                                                                            \
      hipLaunchKernelGGL((k_pqr_step<T, Q, C, true>), dim3(nblocks), dim3(BS), lds, s, d_blk, states, parts,    \
                         total_parts, frop, bmap, active, i, eps, stamp, report, tag);                          \
    else                                                                                                        \
      hipLaunchKernelGGL((k_pqr_step<T, Q, C, false>), dim3(nblocks), dim3(BS), lds, s, d_blk, states, parts,   \
                         total_parts, frop, bmap, active, i, eps, stamp, report, tag);                          \
  } while (0)
  if (cw == PQR_CW) {
    if (!regs)
      SPAQR_PQR_GO(0, PQR_CW / 4);
    else if (rows <= 128)
      SPAQR_PQR_GO(2, PQR_CW / 4);
    else if (rows <= 192)
      SPAQR_PQR_GO(3, PQR_CW / 4);
    else if (rows <= 256)
      SPAQR_PQR_GO(4, PQR_CW / 4);
    else if (rows <= 320)
      SPAQR_PQR_GO(5, PQR_CW / 4);
    else if (rows <= 384)
      SPAQR_PQR_GO(6, PQR_CW / 4);
    else if (rows <= 512)
      SPAQR_PQR_GO(8, PQR_CW / 4);
    else if (rows <= 768)
      SPAQR_PQR_GO(12, PQR_CW / 4);
    else if (rows <= 1024)
      SPAQR_PQR_GO(16, PQR_CW / 4);
    else
      SPAQR_PQR_GO(0, PQR_CW / 4);
  } else {
    throw Error(SPAQR_EARG, "internal: unsupported pivot chunk width");
  }
#undef SPAQR_PQR_GO
  SPAQR_HIP(hipGetLastError());
}

namespace {

// waves of k_pqr_run<T, PQ, NCW> that fit on the device at once (0 without
// cooperative launch support); queried once per kernel
template <typename T, int PQ, int NCW>
int run_capacity() {
  static int cap = -1;
  if (cap < 0) {
    int dev = 0, cus = 0, per = 0, coop = 0;
    SPAQR_HIP(hipGetDevice(&dev));
    SPAQR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SPAQR_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    SPAQR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pqr_run<T, PQ, NCW>, 64, 0));
    cap = coop ? per * cus : 0;
  }
  return cap;
}

template <typename T, int PQ>
int run_capacity_w(int ncw) {
  if (ncw == 8) return run_capacity<T, PQ, 8>();
  if (ncw == 16) return run_capacity<T, PQ, 16>();
  if constexpr (PQ == 2) return run_capacity<T, PQ, 32>();
  return 0;
}

}  // namespace

// Chunk width of the persistent form (columns per wave): the narrowest of 8,
// 16, 32 (16 at most above 128 rows) that keeps every matrix at or below 256
// chunks (at most 512 with the widest), within the co-resident limit and at
// most PQR_RUN_MAX_WAVES waves; 0 when the form does not apply.  The form
// aborted once on a batch of 1805 waves, with no cause found: batches of
// that size take the per-step form until one is.
template <typename T>
int pqr_run_width(int max_m, const std::vector<int>& ns, int* rows) {
  // Opt-in (SPAQR_PQR_PERSISTENT set): the form has not yet run on every
  // workload shape.  SPAQR_NO_COOP (no cooperative launches, for tools that
  // cannot follow them) and SPAQR_PQR_STEPS (one launch per step) keep the
  // other form.
  if (!std::getenv("SPAQR_PQR_PERSISTENT")) return 0;
  if (std::getenv("SPAQR_NO_COOP") || std::getenv("SPAQR_PQR_STEPS")) return 0;
  if (max_m > PQR_RUN_ROWS || ns.empty()) return 0;
  const int pq = max_m <= 128 ? 2 : 4;
  *rows = 64 * pq;
  const int top = pq == 2 ? 32 : 16;  // 32 columns of 256 rows do not fit in registers
  for (int ncw = 8; ncw <= top; ncw *= 2) {
    int64_t total = 0;
    int widest = 0;
    for (int n : ns) {
      const int nb = std::max(1, (n + ncw - 1) / ncw);
      total += nb;
      widest = std::max(widest, nb);
    }
    const int cap = pq == 2 ? run_capacity_w<T, 2>(ncw) : run_capacity_w<T, 4>(ncw);
    if (total <= std::min<int64_t>(cap, PQR_RUN_MAX_WAVES) &&
        (widest <= 256 || (ncw == top && widest <= PQR_POLL * 64)))
      return ncw;
  }
  return 0;
}

template <typename T>
void launch_pqr_run(const PQRDesc* d_desc, int nblocks, const int2* bmap, const PQRXch& xc, double eps, int cw,
                    unsigned long long* stamp, hipStream_t s) {
  if (nblocks <= 0) return;
  if (nblocks != xc.G) throw Error(SPAQR_EARG, "internal: persistent pivoted QR grid mismatch");
  const int pq = xc.rows / 64;
  const void* fn = nullptr;
#define SPAQR_PQR_RUN(Q, C) \
  if (pq == Q && cw == C) fn = reinterpret_cast<const void*>(&k_pqr_run<T, Q, C>);
  SPAQR_PQR_RUN(2, 8)
  SPAQR_PQR_RUN(2, 16)
  SPAQR_PQR_RUN(2, 32)
  SPAQR_PQR_RUN(4, 8)
  SPAQR_PQR_RUN(4, 16)
#undef SPAQR_PQR_RUN
  if (!fn || xc.rows != 64 * pq) throw Error(SPAQR_EARG, "internal: unsupported persistent pivoted QR shape");
  const int cap = pq == 2 ? run_capacity_w<T, 2>(cw) : run_capacity_w<T, 4>(cw);
  if (nblocks > cap) throw Error(SPAQR_EARG, "internal: persistent pivoted QR exceeds the co-resident limit");
  PQRXch x = xc;
  const PQRDesc* dd = d_desc;
  const int2* bm = bmap;
  double e = eps;
  unsigned long long* st = stamp;
  void* args[] = {(void*)&dd, (void*)&bm, (void*)&x, (void*)&e, (void*)&st};
  SPAQR_HIP(hipLaunchCooperativeKernel(fn, dim3(nblocks), dim3(64), args, 0, s));
}

template <typename T>
void launch_pqr_finish(const PQRDesc* d_desc, int nmat, PQRState* states, int steps, hipStream_t s) {
  if (nmat <= 0) return;
  hipLaunchKernelGGL(k_pqr_finish<T>, dim3(nmat), dim3(BS), 0, s, d_desc, (const PQRState*)states, steps);
  SPAQR_HIP(hipGetLastError());
}

#define SPAQR_PQR_INST(T)                                                                             \
  template void launch_pqr_init<T>(const PQRDesc*, int, PQRState*, PQRPart*, double*, const int2*, hipStream_t); \
  template void launch_pqr_step<T>(const PQRDesc*, int, int, PQRState*, PQRPart*, const double*, const int2*,  \
                                   int*, int, double, int, int, int, unsigned long long*,                     \
                                   unsigned long long*, unsigned, bool, hipStream_t);                         \
  template void launch_pqr_finish<T>(const PQRDesc*, int, PQRState*, int, hipStream_t);                   \
  template int pqr_run_width<T>(int, const std::vector<int>&, int*);                                     \
  template void launch_pqr_run<T>(const PQRDesc*, int, const int2*, const PQRXch&, double, int,            \
                                  unsigned long long*, hipStream_t);

SPAQR_PQR_INST(double)
SPAQR_PQR_INST(float)

}  // namespace spaqr
