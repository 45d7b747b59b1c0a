// Device kernels of the spaQR factorization for gfx950 (wave64).
//
//  - gather / scatter of row groups into dense fronts (Section 2.3 fronts,
//    Section 2.4 scaling blocks, Section 2.5.2 [A_np^T A_p1n] blocks);
//  - batched blocked Householder QR (panel + compact-WY trailing update),
//    reflector convention beta = -sign(alpha)||x||, sign(0) = +1;
//  - batched column-pivoted QR stopped by |R_ii| >= eps |R_11| (Section 4),
//    FP64 column norms with the downdate / recompute rule of LAPACK Working
//    Note 176;
//  - batched right triangular solves (scaling, Section 2.4), owner selection
//    of reassigned rows (Section 2.3), row copies, identity writes.
#include <hip/hip_runtime.h>

#include <climits>

#include <cfloat>
#include <cmath>

#include "spaqr_impl.h"
#include "wave.h"

namespace spaqr {

namespace {

constexpr int BS = 256;

template <typename T>
struct Unit;
template <>
struct Unit<double> {
  static constexpr double u = DBL_EPSILON / 2;
};
template <>
struct Unit<float> {
  static constexpr double u = FLT_EPSILON / 2;
};

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

// Sum over the 256 threads of a block; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ---------------------------------------------------------------------------
// gather
// ---------------------------------------------------------------------------
constexpr int GATHER_COLS = 16;

template <typename T>
__global__ __launch_bounds__(BS) void k_gather(const GatherDesc* __restrict__ D) {
  const GatherDesc d = D[blockIdx.x];
  const int c0 = blockIdx.y * GATHER_COLS;
  if (c0 >= d.ncols) return;
  const int c1 = min(d.ncols, c0 + GATHER_COLS);
  const T* src = static_cast<const T*>(d.src);
  T* dst = static_cast<T*>(d.dst);
  // a thread's rows of all the block's columns are loaded before any store
  int sc[GATHER_COLS];
#pragma unroll
  for (int u = 0; u < GATHER_COLS; ++u) sc[u] = c0 + u < c1 ? d.colmap[c0 + u] : -1;
  for (int r = threadIdx.x; r < d.nrows; r += BS) {
    T v[GATHER_COLS];
#pragma unroll
    for (int u = 0; u < GATHER_COLS; ++u) v[u] = sc[u] >= 0 ? src[r + (int64_t)sc[u] * d.src_ld] : T(0);
    if (!d.transpose) {
#pragma unroll
      for (int u = 0; u < GATHER_COLS; ++u)
        if (c0 + u < c1) dst[d.row0 + r + (d.col0 + c0 + u) * d.dst_ld] = v[u];
    } else {
#pragma unroll
      for (int u = 0; u < GATHER_COLS; ++u)
        if (c0 + u < c1) dst[c0 + u + (d.col0 + r) * d.dst_ld] = v[u];
    }
  }
}

// one work-group per map: clear, then place the group's columns
__global__ __launch_bounds__(BS) void k_expand_maps(const ExpandDesc* __restrict__ D) {
  const ExpandDesc d = D[blockIdx.x];
  for (int c = threadIdx.x; c < d.n; c += BS) d.out[c] = -1;
  __syncthreads();
  for (int i = threadIdx.x; i < d.nslots; i += BS) {
    const int c = d.fpos[i];
    if (c >= 0 && c < d.n) d.out[c] = i;
  }
}

template <typename T>
__global__ void k_scatter_csr(T* __restrict__ base, const int64_t* __restrict__ dst,
                              const double* __restrict__ val, int64_t nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) base[dst[e]] = static_cast<T>(val[e]);
}

// ---------------------------------------------------------------------------
// B <- B R^-1 (R upper triangular).  One thread per row of B, grid over
// (descriptor, chunk of BS rows).  Columns are solved left-looking in
// register blocks of TRSM_NB: the block's entries are loaded, reduced by
// the already solved columns (re-read from B, coalesced over rows), then
// solved in registers.  R is read at block-uniform addresses.
// ---------------------------------------------------------------------------
constexpr int TRSM_NB = 16;

template <typename T>
__global__ __launch_bounds__(BS) void k_trsm(const TrsmDesc* __restrict__ D) {
  const TrsmDesc d = D[blockIdx.x];
  if ((int)blockIdx.y * BS >= d.nrows) return;  // whole block
  const int r = blockIdx.y * BS + threadIdx.x;
  const bool live = r < d.nrows;
  T* B = static_cast<T*>(d.B);
  const T* R = static_cast<const T*>(d.R);
  for (int jb = 0; jb < d.c; jb += TRSM_NB) {
    const int nb = min(TRSM_NB, d.c - jb);
    double acc[TRSM_NB];
#pragma unroll
    for (int k = 0; k < TRSM_NB; ++k)
      acc[k] = (live && k < nb) ? (double)B[r + (int64_t)d.colmap[jb + k] * d.ldb] : 0.0;
    for (int i = 0; i < jb; ++i) {
      const double bi = live ? (double)B[r + (int64_t)d.colmap[i] * d.ldb] : 0.0;
      const T* ri = R + i + (int64_t)jb * d.ldr;
#pragma unroll
      for (int k = 0; k < TRSM_NB; ++k)
        if (k < nb) acc[k] -= bi * (double)ri[k * d.ldr];
    }
#pragma unroll
    for (int k = 0; k < TRSM_NB; ++k) {
      if (k < nb) {
        const T* rk = R + (jb + k) + (int64_t)jb * d.ldr;
        acc[k] /= (double)rk[k * d.ldr];
#pragma unroll
        for (int k2 = k + 1; k2 < TRSM_NB; ++k2)
          if (k2 < nb) acc[k2] -= acc[k] * (double)rk[k2 * d.ldr];
      }
    }
    if (live) {
#pragma unroll
      for (int k = 0; k < TRSM_NB; ++k)
        if (k < nb) B[r + (int64_t)d.colmap[jb + k] * d.ldb] = static_cast<T>(acc[k]);
    }
  }
}

// Same solve with the work-group's 64 rows of B held in LDS (FP64) while
// they are solved: B is read and written once, the left-looking updates
// read the solved columns from LDS, and the current 16-column block of R is
// staged in LDS.  One wave per work-group, thread = row.  Dynamic LDS:
// c (64 + 1 + TRSM_NB) doubles for the largest c of the launch.  The grid
// is one work-group per (descriptor, 64-row block) pair that exists, listed
// in bmap, so short descriptors of a launch start no idle work-groups.
template <typename T>
__global__ __launch_bounds__(TRSM_ROWS) void k_trsm_lds(const TrsmDesc* __restrict__ D,
                                                        const int2* __restrict__ bmap, int cmax) {
  extern __shared__ double lds[];
  const int2 bm = bmap[blockIdx.x];
  const TrsmDesc d = D[bm.x];
  if (bm.y * TRSM_ROWS >= d.nrows) return;  // whole block (not listed by the launcher)
  double* Xs = lds;                                        // [c][TRSM_ROWS + 1]
  double* Rs = lds + (size_t)cmax * (TRSM_ROWS + 1);       // [c][TRSM_NB]
  const int lane = threadIdx.x;
  const int r = bm.y * TRSM_ROWS + lane;
  const bool live = r < d.nrows;
  T* B = static_cast<T*>(d.B);
  const T* R = static_cast<const T*>(d.R);
  const int c = d.c;
  for (int j = 0; j < c; ++j)
    Xs[j * (TRSM_ROWS + 1) + lane] = live ? (double)B[r + (int64_t)d.colmap[j] * d.ldb] : 0.0;
  for (int jb = 0; jb < c; jb += TRSM_NB) {
    const int nb = min(TRSM_NB, c - jb);
    __syncthreads();
    for (int e = lane; e < (jb + nb) * TRSM_NB; e += TRSM_ROWS) {
      const int i = e / TRSM_NB, k = e % TRSM_NB;
      Rs[e] = k < nb ? (double)R[i + (int64_t)(jb + k) * d.ldr] : 0.0;
    }
    __syncthreads();
    double acc[TRSM_NB];
#pragma unroll
    for (int k = 0; k < TRSM_NB; ++k) acc[k] = k < nb ? Xs[(jb + k) * (TRSM_ROWS + 1) + lane] : 0.0;
    for (int i = 0; i < jb; ++i) {
      const double bi = Xs[i * (TRSM_ROWS + 1) + lane];
#pragma unroll
      for (int k = 0; k < TRSM_NB; ++k) acc[k] -= bi * Rs[i * TRSM_NB + k];
    }
#pragma unroll
    for (int k = 0; k < TRSM_NB; ++k) {
      if (k < nb) {
        acc[k] /= Rs[(jb + k) * TRSM_NB + k];
#pragma unroll
        for (int k2 = k + 1; k2 < TRSM_NB; ++k2)
          if (k2 < nb) acc[k2] -= acc[k] * Rs[(jb + k) * TRSM_NB + k2];
      }
    }
#pragma unroll
    for (int k = 0; k < TRSM_NB; ++k)
      if (k < nb) Xs[(jb + k) * (TRSM_ROWS + 1) + lane] = acc[k];
  }
  if (live)
    for (int j = 0; j < c; ++j) B[r + (int64_t)d.colmap[j] * d.ldb] = static_cast<T>(Xs[j * (TRSM_ROWS + 1) + lane]);
}

// owner of each row: cluster with the largest sum of squared entries, the
// first (lowest) cluster on ties.  A work-group covers 64 rows (one per
// lane, coalesced column reads); its 4 waves take every 4th cluster and
// their best (value, cluster) pairs are merged in LDS.
template <typename T>
__global__ __launch_bounds__(BS) void k_owner(const OwnerDesc* __restrict__ D) {
  const OwnerDesc d = D[blockIdx.x];
  const T* A = static_cast<const T*>(d.A);
  const int nrows = d.nrows_dev ? d.nrows_dev[0] : d.nrows;
  const int r0 = blockIdx.y * 64;
  if (r0 >= nrows) return;  // uniform over the block
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = r0 + lane;
  __shared__ double sv[4][64];
  __shared__ int sq[4][64];
  int best = INT_MAX;
  double bv = -1.0;
  if (r < nrows)
    for (int q = wv; q < d.ncl; q += 4) {
      // 16 columns per pass: indices, then entries, then the sum in column order
      const int cb = d.cl_off[q], ce = d.cl_off[q + 1];
      double s = 0.0;
#pragma unroll 1
      for (int c = cb; c < ce; c += 16) {
        int cm[16];
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) cm[u] = d.colmap[min(c + u, ce - 1)];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = A[r + (int64_t)cm[u] * d.lda];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (c + u < ce) s += (double)v[u] * (double)v[u];
      }
      if (s > bv) bv = s, best = q;
    }
  sv[wv][lane] = bv;
  sq[wv][lane] = best;
  __syncthreads();
  if (wv == 0 && r < nrows) {
    for (int w = 1; w < 4; ++w)
      if (sv[w][lane] > bv || (sv[w][lane] == bv && sq[w][lane] < best)) bv = sv[w][lane], best = sq[w][lane];
    d.owner[r] = best == INT_MAX ? 0 : best;
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_rowcopy(const RowCopyDesc* __restrict__ D) {
  const RowCopyDesc d = D[blockIdx.x];
  const int c0 = blockIdx.y * GATHER_COLS;
  if (c0 >= d.ncols) return;
  const int c1 = min(d.ncols, c0 + GATHER_COLS);
  const T* src = static_cast<const T*>(d.src);
  T* dst = static_cast<T*>(d.dst);
  for (int c = c0; c < c1; ++c)
    for (int i = threadIdx.x; i < d.nrows; i += BS) {
      const int sr = d.rows[i];
      const bool z = d.tri && c < sr - d.tri_base;
      dst[i + c * d.dst_ld] = z ? T(0) : src[sr + c * d.src_ld];
    }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_extract(const ExtractDesc* __restrict__ D) {
  const ExtractDesc d = D[blockIdx.x];
  T* A = static_cast<T*>(d.A);
  T* R = static_cast<T*>(d.R);
  __shared__ double sh[4];
  double fro = 0.0;
  double mn = DBL_MAX;
  for (int j = 0; j < d.c; ++j)
    for (int i = threadIdx.x; i < d.c; i += BS) {
      T* a = A + i + j * d.lda;
      const T v = i <= j ? *a : T(0);
      R[i + j * d.ldr] = v;
      fro += (double)v * (double)v;
      if (i == j) mn = fmin(mn, fabs((double)v));
      *a = i == j ? T(1) : T(0);
    }
  fro = block_sum(fro, sh);
  // min over the block
  double m2 = mn;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m2 = fmin(m2, __shfl_xor(m2, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m2;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mm = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
    d.flag[0] = mm <= 64.0 * Unit<T>::u * sqrt(fro) ? 1 : 0;
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_scatter(const ScatterDesc* __restrict__ D) {
  const ScatterDesc d = D[blockIdx.x];
  const int rk = d.rank[0];
  const T* C = static_cast<const T*>(d.C);
  T* dst = static_cast<T*>(d.dst);
  if (d.transpose) {
    // dst[r + colmap[i] * ld] = C[i + (col0 + r) * ldc]
    for (int i = blockIdx.y; i < rk; i += gridDim.y)
      for (int r = threadIdx.x; r < d.nrows; r += BS)
        dst[r + (int64_t)d.colmap[i] * d.ld] = C[i + (d.col0 + r) * d.ldc];
  } else if (d.identity) {
    for (int j = blockIdx.y; j < rk; j += gridDim.y)
      for (int i = threadIdx.x; i < rk; i += BS) dst[i + (int64_t)d.colmap[j] * d.ld] = i == j ? T(1) : T(0);
  } else {
    for (int c = blockIdx.y; c < d.ncols; c += gridDim.y)
      for (int i = threadIdx.x; i < rk; i += BS)
        dst[i + (int64_t)d.colmap[c] * d.ld] = C[i + (d.col0 + c) * d.ldc];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
void launch_gather(const GatherDesc* d_desc, int n, int max_cols, hipStream_t s) {
  if (n <= 0 || max_cols <= 0) return;
  dim3 grid(n, (max_cols + GATHER_COLS - 1) / GATHER_COLS);
  hipLaunchKernelGGL(k_gather<T>, grid, dim3(BS), 0, s, d_desc);
  SPAQR_HIP(hipGetLastError());
}

void launch_expand_maps(const ExpandDesc* d_desc, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_expand_maps, dim3(n), dim3(BS), 0, s, d_desc);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_scatter_csr(T* base, const int64_t* dst, const double* ahat, int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_scatter_csr<T>, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, base, dst,
                     ahat, nnz);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_trsm(const TrsmDesc* d_desc, int n, int max_rows, int max_c, const int2* d_rowblocks,
                 int n_rowblocks, hipStream_t s) {
  if (n <= 0 || max_rows <= 0) return;
  static int lds_cap = -1;
  if (lds_cap < 0) {
    int dev = 0;
    SPAQR_HIP(hipGetDevice(&dev));
    SPAQR_HIP(hipDeviceGetAttribute(&lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  }
  const size_t lds = (size_t)max_c * (TRSM_ROWS + 1 + TRSM_NB) * sizeof(double);
  if (max_c > 0 && lds <= (size_t)lds_cap) {
    if (n_rowblocks <= 0) return;
    hipLaunchKernelGGL(k_trsm_lds<T>, dim3(n_rowblocks), dim3(TRSM_ROWS), lds, s, d_desc, d_rowblocks, max_c);
  } else {
    hipLaunchKernelGGL(k_trsm<T>, dim3(n, (max_rows + BS - 1) / BS), dim3(BS), 0, s, d_desc);
  }
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_owner(const OwnerDesc* d_desc, int n, int max_rows, hipStream_t s) {
  if (n <= 0 || max_rows <= 0) return;
  hipLaunchKernelGGL(k_owner<T>, dim3(n, (max_rows + 63) / 64), dim3(BS), 0, s, d_desc);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_rowcopy(const RowCopyDesc* d_desc, int n, int max_cols, hipStream_t s) {
  if (n <= 0 || max_cols <= 0) return;
  hipLaunchKernelGGL(k_rowcopy<T>, dim3(n, (max_cols + GATHER_COLS - 1) / GATHER_COLS), dim3(BS), 0, s,
                     d_desc);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_extract(const ExtractDesc* d_desc, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_extract<T>, dim3(n), dim3(BS), 0, s, d_desc);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_scatter(const ScatterDesc* d_desc, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter<T>, dim3(n, 64), dim3(BS), 0, s, d_desc);
  SPAQR_HIP(hipGetLastError());
}

#define SPAQR_INST(T)                                                                          \
  template void launch_gather<T>(const GatherDesc*, int, int, hipStream_t);                    \
  template void launch_scatter_csr<T>(T*, const int64_t*, const double*, int64_t, hipStream_t); \
  template void launch_trsm<T>(const TrsmDesc*, int, int, int, const int2*, int, hipStream_t);                        \
  template void launch_owner<T>(const OwnerDesc*, int, int, hipStream_t);                           \
  template void launch_rowcopy<T>(const RowCopyDesc*, int, int, hipStream_t);                         \
  template void launch_extract<T>(const ExtractDesc*, int, hipStream_t);                       \
  template void launch_scatter<T>(const ScatterDesc*, int, hipStream_t);

SPAQR_INST(double)
SPAQR_INST(float)

}  // namespace spaqr
