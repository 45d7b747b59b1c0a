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
// eps |R_00|, or at or below the numerical-rank floor noise * ||A||_F, or
// when `forced` steps were taken.  Pivot ties go to the lowest column index.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

#include "spaqr_impl.h"

namespace spaqr {

namespace {

constexpr int BS = 256;
constexpr int PL = 6;  // chunk partials per thread fetched up front
static_assert(PQR_CW == 8, "a pivot step gives each of its 4 waves cw/4 columns");

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// block-wide argmax of (val, idx): larger val wins, lowest idx on ties
__device__ __forceinline__ void block_argmax(double& bv, int& bi, double* shv, int* shi) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > bv || (ov == bv && oi < bi)) bv = ov, bi = oi;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) shv[threadIdx.x >> 6] = bv, shi[threadIdx.x >> 6] = bi;
  __syncthreads();
  bv = shv[0];
  bi = shi[0];
  for (int w = 1; w < 4; ++w)
    if (shv[w] > bv || (shv[w] == bv && shi[w] < bi)) bv = shv[w], bi = shi[w];
}

__device__ __forceinline__ void house_scalars(double alpha, double xn2, double& beta, double& tau,
                                              double& scal) {
  if (xn2 == 0.0) {
    beta = alpha;
    tau = 0.0;
    scal = 1.0;
  } else {
    const double s = alpha < 0.0 ? -1.0 : 1.0;
    beta = -s * sqrt(alpha * alpha + xn2);
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
                                                 const int2* __restrict__ bmap) {
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
    p.fro = fro;
    p.idx = bi;
    p.pad_ = 0;
    parts[d.blk0 + bm.y] = p;
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
// launcher picks 2 or 4 when that covers the batch's tallest matrix; 0
// keeps the columns in memory, which measured faster for taller ones).
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

template <typename T, int PQ, int NC>
__global__ __launch_bounds__(BS) void k_pqr_step(const PQRDesc* __restrict__ D, PQRState* __restrict__ S,
                                                 PQRPart* __restrict__ parts, int total_parts,
                                                 const int2* __restrict__ bmap, int* __restrict__ active,
                                                 int i, double eps, unsigned long long* stamp) {
  const StampScope timing(stamp);
  extern __shared__ double x[];  // pivot column rows i..m-1
  __shared__ double sh[4];
  __shared__ double shv[4];
  __shared__ int shi[4];
  // Loads are issued in the order they are needed (they complete in
  // order): block map with the first descriptor (most batches of single
  // large matrices need no second round trip), state and chunk partials,
  // then this work-group's own columns, which are consumed last.
  const int2 bm = bmap[blockIdx.x];
  const PQRDesc d0 = D[0];
  const int mi = bm.x, ch = bm.y;
  const PQRDesc d = mi == 0 ? d0 : D[mi];
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
  double pval[PL];
  int pidx[PL];
  double pfro[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int k = tid + u * BS;
    if (k < d.nblk) {
      const PQRPart q = prd[d.blk0 + k];
      pval[u] = q.val, pidx[u] = q.idx, pfro[u] = q.fro;
    } else {
      pval[u] = -1.0, pidx[u] = INT_MAX, pfro[u] = 0.0;
    }
  }
  const bool regs = PQ > 0 && m - i <= 64 * PQ;
  int jcol[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) jcol[k] = c0 + wv + 4 * k;
  double yv[NC][PQ > 0 ? PQ : 1];
  double v1p[NC], v2p[NC], dnp[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) v1p[k] = 0.0, v2p[k] = 1.0, dnp[k] = 1.0;
  if (regs) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int j = jcol[k] < c1 ? jcol[k] : c0;
      const T* y = A + (int64_t)j * lda;
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int r = i + lane + 64 * q;
        yv[k][q] = r < m ? (double)y[r] : 0.0;
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
  double bv = -1.0, fro = 0.0;
  int bi = INT_MAX;
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    if (pval[u] > bv || (pval[u] == bv && pidx[u] < bi)) bv = pval[u], bi = pidx[u];
    fro += pfro[u];
  }
  for (int k = tid + PL * BS; k < d.nblk; k += BS) {
    const PQRPart q = prd[d.blk0 + k];
    if (q.val > bv || (q.val == bv && q.idx < bi)) bv = q.val, bi = q.idx;
    fro += q.fro;
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
    else if (i > 0)
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
          const int r = i + lane + 64 * q;
          if (r < m) dot += x[r - i] * yv[k][q];
        }
      dot = wave_sum(dot);
      const double f = tv * dot;
      const double yi = __shfl(yv[k][0], 0, 64) - f;
      if (tv != 0.0)
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int r = i + lane + 64 * q;
          if (r < m) {
            const T nv = static_cast<T>(yv[k][q] - f * x[r - i]);
            y[r] = nv;
            yv[k][q] = (double)nv;
          }
        }
      const double v1 = v1p[k];
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
            const int r = i + lane + 64 * q;
            if (r > i && r < m) s2 += yv[k][q] * yv[k][q];
          }
          s2 = sqrt(wave_sum(s2));
          if (lane == 0) vn1[j] = s2, vn2[j] = s2;
        } else if (lane == 0) {
          vn1[j] = v1 * sqrt(temp);
        }
      }
    }
  }
  for (int j = c0 + wv; !regs && j < c1; j += 4) {
    if (j == p || done[j] != 0.0) continue;
    T* y = A + (int64_t)j * lda;
    double dot = 0.0;
    if (tv != 0.0)
      for (int r = i + lane; r < m; r += 64) dot += x[r - i] * (double)y[r];
    dot = wave_sum(dot);
    const double f = tv * dot;
    const double yi = (double)y[i] - f;
    if (tv != 0.0)
      for (int r = i + lane; r < m; r += 64) y[r] = static_cast<T>((double)y[r] - f * x[r - i]);
    const double v1 = vn1[j];
    if (v1 != 0.0) {
      const double ay = fabs((double)static_cast<T>(yi));
      double temp = 1.0 - (ay / v1) * (ay / v1);
      temp = temp > 0.0 ? temp : 0.0;
      const double ratio = v1 / vn2[j];
      const double temp2 = temp * ratio * ratio;
      if (temp2 <= tol3z) {
        double s = 0.0;
        for (int r = i + 1 + lane; r < m; r += 64) s += (double)y[r] * (double)y[r];
        s = sqrt(wave_sum(s));
        if (lane == 0) vn1[j] = s, vn2[j] = s;
      } else if (lane == 0) {
        vn1[j] = v1 * sqrt(temp);
      }
    }
  }
  if (tid == 0 && p >= c0 && p < c1) done[p] = 1.0;
  __syncthreads();
  chunk_argmax(vn1, done, c0, c1, p, bv, bi, shv, shi);
  if (tid == 0) {
    PQRPart q;
    q.val = bv;
    q.fro = 0.0;
    q.idx = bi;
    q.pad_ = 0;
    pwr[d.blk0 + ch] = q;
  }
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
void launch_pqr_init(const PQRDesc* d_desc, int nblocks, PQRState* states, PQRPart* parts,
                     const int2* bmap, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_pqr_init<T>, dim3(nblocks), dim3(BS), 0, s, d_desc, states, parts, bmap);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_pqr_step(const PQRDesc* d_desc, int nblocks, int total_parts, PQRState* states,
                     PQRPart* parts, const int2* bmap, int* active, int i, double eps, int max_m, int cw,
                     unsigned long long* stamp, hipStream_t s) {
  if (nblocks <= 0) return;
  const size_t lds = (size_t)std::max(1, max_m) * sizeof(double);
  if (lds > 64 * 1024) throw Error(SPAQR_EARG, "rank-revealing QR block taller than 8192 rows");
  const int rows = max_m - i;
#define SPAQR_PQR_GO(Q, C)                                                                                   \
  hipLaunchKernelGGL((k_pqr_step<T, Q, C>), dim3(nblocks), dim3(BS), lds, s, d_desc, states, parts, total_parts, \
                     bmap, active, i, eps, stamp)
  if (cw == PQR_CW) {
    if (rows <= 128)
      SPAQR_PQR_GO(2, PQR_CW / 4);
    else if (rows <= 256)
      SPAQR_PQR_GO(4, PQR_CW / 4);
    else
      SPAQR_PQR_GO(0, PQR_CW / 4);
  } else {
    throw Error(SPAQR_EARG, "internal: unsupported pivot chunk width");
  }
#undef SPAQR_PQR_GO
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_pqr_finish(const PQRDesc* d_desc, int nmat, PQRState* states, int steps, hipStream_t s) {
  if (nmat <= 0) return;
  hipLaunchKernelGGL(k_pqr_finish<T>, dim3(nmat), dim3(BS), 0, s, d_desc, (const PQRState*)states, steps);
  SPAQR_HIP(hipGetLastError());
}

#define SPAQR_PQR_INST(T)                                                                             \
  template void launch_pqr_init<T>(const PQRDesc*, int, PQRState*, PQRPart*, const int2*, hipStream_t); \
  template void launch_pqr_step<T>(const PQRDesc*, int, int, PQRState*, PQRPart*, const int2*, int*, int, \
                                   double, int, int, unsigned long long*, hipStream_t);               \
  template void launch_pqr_finish<T>(const PQRDesc*, int, PQRState*, int, hipStream_t);

SPAQR_PQR_INST(double)
SPAQR_PQR_INST(float)

}  // namespace spaqr
