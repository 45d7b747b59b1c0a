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

#include <cfloat>
#include <cmath>

#include "spaqr_impl.h"

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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 256 threads of a block; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Householder scalars for x = [alpha; tail], ||tail||^2 = xn2.
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
  if (!d.transpose) {
    for (int c = c0; c < c1; ++c) {
      const int sc = d.colmap[c];
      T* out = dst + d.row0 + (d.col0 + c) * d.dst_ld;
      if (sc >= 0) {
        const T* in = src + (int64_t)sc * d.src_ld;
        for (int r = threadIdx.x; r < d.nrows; r += BS) out[r] = in[r];
      } else {
        for (int r = threadIdx.x; r < d.nrows; r += BS) out[r] = T(0);
      }
    }
  } else {
    for (int c = c0; c < c1; ++c) {
      const int sc = d.colmap[c];
      T* out = dst + c + d.col0 * d.dst_ld;
      if (sc >= 0) {
        const T* in = src + (int64_t)sc * d.src_ld;
        for (int r = threadIdx.x; r < d.nrows; r += BS) out[r * d.dst_ld] = in[r];
      } else {
        for (int r = threadIdx.x; r < d.nrows; r += BS) out[r * d.dst_ld] = T(0);
      }
    }
  }
}

template <typename T>
__global__ void k_scatter_csr(T* __restrict__ base, const int64_t* __restrict__ dst,
                              const double* __restrict__ val, int64_t nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) base[dst[e]] = static_cast<T>(val[e]);
}

// ---------------------------------------------------------------------------
// blocked Householder QR
// ---------------------------------------------------------------------------
constexpr int QR_NB = 32;
constexpr int QR_TN = 64;

// Factor columns [j0, j0+kb) of every matrix (rows j0..m-1) and build the
// triangular factor T of the compact-WY form Q = I - V T V^T.
template <typename T>
__global__ __launch_bounds__(BS) void k_qr_panel(const QRDesc* __restrict__ D, int j0,
                                                 double* __restrict__ tbuf) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(QR_NB, kk - j0);
  T* A = static_cast<T*>(d.A);
  T* tau = static_cast<T*>(d.tau);
  const int64_t lda = d.lda;
  const int m = d.m;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  __shared__ double sh[4];
  __shared__ double s_tau[QR_NB];
  __shared__ double G[QR_NB][QR_NB + 1];

  for (int i = 0; i < kb; ++i) {
    const int c = j0 + i;
    T* col = A + c * lda;
    double part = 0.0;
    for (int r = c + 1 + tid; r < m; r += BS) {
      const double v = col[r];
      part += v * v;
    }
    const double xn2 = block_sum(part, sh);
    const double alpha = col[c];
    double beta, tv, scal;
    house_scalars(alpha, xn2, beta, tv, scal);
    if (tv != 0.0)
      for (int r = c + 1 + tid; r < m; r += BS) col[r] = static_cast<T>(col[r] * scal);
    __syncthreads();
    if (tv != 0.0) {
      for (int cc = c + 1 + wv; cc < j0 + kb; cc += 4) {
        T* y = A + cc * lda;
        const double yc = y[c];
        double dot = 0.0;
        for (int r = c + 1 + lane; r < m; r += 64) dot += (double)col[r] * (double)y[r];
        dot = wave_sum(dot) + yc;
        const double f = tv * dot;
        if (lane == 0) y[c] = static_cast<T>(yc - f);
        for (int r = c + 1 + lane; r < m; r += 64) y[r] = static_cast<T>(y[r] - f * (double)col[r]);
      }
    }
    __syncthreads();
    if (tid == 0) {
      col[c] = static_cast<T>(beta);
      tau[c] = static_cast<T>(tv);
      s_tau[i] = static_cast<double>(static_cast<T>(tv));
    }
    __syncthreads();
  }
  // G[a][b] = v_a^T v_b for a < b (v_a has a unit entry at row j0+a)
  for (int pr = wv; pr < kb * kb; pr += 4) {
    const int a = pr / kb, b = pr % kb;
    if (a >= b) continue;
    const T* va = A + (j0 + a) * lda;
    const T* vb = A + (j0 + b) * lda;
    double dot = 0.0;
    for (int r = j0 + b + 1 + lane; r < m; r += 64) dot += (double)va[r] * (double)vb[r];
    dot = wave_sum(dot);
    if (lane == 0) G[a][b] = dot + (double)va[j0 + b];
  }
  __syncthreads();
  if (tid == 0) {
    double* Tm = tbuf + (int64_t)blockIdx.x * QR_NB * QR_NB;
    for (int i = 0; i < kb; ++i) {
      Tm[i * QR_NB + i] = s_tau[i];
      for (int a = 0; a < i; ++a) {
        double acc = 0.0;
        for (int b = a; b < i; ++b) acc += Tm[a * QR_NB + b] * G[b][i];
        Tm[a * QR_NB + i] = -s_tau[i] * acc;
      }
      for (int a = i + 1; a < QR_NB; ++a) Tm[a * QR_NB + i] = 0.0;
    }
  }
}

// C <- (I - V T V^T)^T C on a tile of QR_TN trailing columns.
template <typename T>
__global__ __launch_bounds__(BS) void k_qr_update(const QRDesc* __restrict__ D, int j0,
                                                  const double* __restrict__ tbuf) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(QR_NB, kk - j0);
  const int c0 = j0 + kb + blockIdx.y * QR_TN;
  if (c0 >= d.n) return;
  const int nc = min(QR_TN, d.n - c0);
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int m = d.m;
  const int tid = threadIdx.x;
  __shared__ double W[QR_NB][QR_TN + 1];
  __shared__ T Vs[32][QR_NB + 1];
  __shared__ T Cs[32][QR_TN + 1];
  const double* Tm = tbuf + (int64_t)blockIdx.x * QR_NB * QR_NB;

  // phase 1: W = V^T C   (thread -> a = tid>>3, columns cg*8 .. cg*8+7)
  const int pa = tid >> 3, pcg = tid & 7;
  double acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;
  for (int r0 = j0; r0 < m; r0 += 32) {
    for (int e = tid; e < 32 * QR_NB; e += BS) {
      const int rr = e & 31, a = e >> 5;
      const int r = r0 + rr;
      T v = T(0);
      if (a < kb && r < m) {
        if (r == j0 + a)
          v = T(1);
        else if (r > j0 + a)
          v = A[r + (j0 + a) * lda];
      }
      Vs[rr][a] = v;
    }
    for (int e = tid; e < 32 * QR_TN; e += BS) {
      const int rr = e & 31, cc = e >> 5;
      const int r = r0 + rr;
      Cs[rr][cc] = (r < m && cc < nc) ? A[r + (c0 + cc) * lda] : T(0);
    }
    __syncthreads();
    if (pa < kb) {
      const int rmax = min(32, m - r0);
      for (int rr = 0; rr < rmax; ++rr) {
        const double v = Vs[rr][pa];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += v * (double)Cs[rr][pcg * 8 + j];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) W[pa][pcg * 8 + j] = acc[j];
  __syncthreads();
  // phase 2: W <- T^T W
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double s = 0.0;
    if (pa < kb)
      for (int a = 0; a <= pa; ++a) s += Tm[a * QR_NB + pa] * W[a][pcg * 8 + j];
    acc[j] = s;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) W[pa][pcg * 8 + j] = acc[j];
  __syncthreads();
  // phase 3: C -= V W   (thread -> row rr = tid & 31, columns cg*8..)
  const int rr = tid & 31, cg = tid >> 5;
  for (int r0 = j0; r0 < m; r0 += 32) {
    for (int e = tid; e < 32 * QR_NB; e += BS) {
      const int r2 = e & 31, a = e >> 5;
      const int r = r0 + r2;
      T v = T(0);
      if (a < kb && r < m) {
        if (r == j0 + a)
          v = T(1);
        else if (r > j0 + a)
          v = A[r + (j0 + a) * lda];
      }
      Vs[r2][a] = v;
    }
    __syncthreads();
    const int r = r0 + rr;
    if (r < m) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int cc = cg * 8 + j;
        if (cc < nc) {
          double s = 0.0;
          for (int a = 0; a < kb; ++a) s += (double)Vs[rr][a] * W[a][cc];
          T* p = A + r + (c0 + cc) * lda;
          *p = static_cast<T>(*p - s);
        }
      }
    }
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// B <- B R^-1 (R upper triangular), rows in parallel
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BS) void k_trsm(const TrsmDesc* __restrict__ D) {
  const TrsmDesc d = D[blockIdx.x];
  T* B = static_cast<T*>(d.B);
  const T* R = static_cast<const T*>(d.R);
  for (int r = threadIdx.x; r < d.nrows; r += BS) {
    for (int j = 0; j < d.c; ++j) {
      T* bj = B + r + (int64_t)d.colmap[j] * d.ldb;
      double acc = *bj;
      const T* rc = R + (int64_t)j * d.ldr;
      for (int i = 0; i < j; ++i) acc -= (double)B[r + (int64_t)d.colmap[i] * d.ldb] * (double)rc[i];
      *bj = static_cast<T>(acc / (double)rc[j]);
    }
  }
}

// owner of each row: cluster with the largest sum of squared entries
template <typename T>
__global__ __launch_bounds__(BS) void k_owner(const OwnerDesc* __restrict__ D) {
  const OwnerDesc d = D[blockIdx.x];
  const T* A = static_cast<const T*>(d.A);
  const int nrows = d.nrows_dev ? d.nrows_dev[0] : d.nrows;
  for (int r = threadIdx.x; r < nrows; r += BS) {
    int best = 0;
    double bv = -1.0;
    for (int q = 0; q < d.ncl; ++q) {
      double s = 0.0;
      for (int c = d.cl_off[q]; c < d.cl_off[q + 1]; ++c) {
        const double v = A[r + (int64_t)d.colmap[c] * d.lda];
        s += v * v;
      }
      if (s > bv) bv = s, best = q;
    }
    d.owner[r] = best;
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

template <typename T>
void launch_scatter_csr(T* base, const int64_t* dst, const double* ahat, int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(k_scatter_csr<T>, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, base, dst,
                     ahat, nnz);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_qr(const QRDesc* d_desc, const std::vector<QRDesc>& h, double* tbuf, hipStream_t s,
               int* launches) {
  if (h.empty()) return;
  int kmax = 0;
  for (auto& d : h) kmax = std::max(kmax, std::min(d.m, d.k));
  for (int j0 = 0; j0 < kmax; j0 += QR_NB) {
    int tiles = 0;
    for (auto& d : h) {
      const int kk = std::min(d.m, d.k);
      if (j0 >= kk) continue;
      const int kb = std::min(QR_NB, kk - j0);
      const int rest = d.n - j0 - kb;
      if (rest > 0) tiles = std::max(tiles, (rest + QR_TN - 1) / QR_TN);
    }
    hipLaunchKernelGGL(k_qr_panel<T>, dim3((unsigned)h.size()), dim3(BS), 0, s, d_desc, j0, tbuf);
    SPAQR_HIP(hipGetLastError());
    ++*launches;
    if (tiles > 0) {
      hipLaunchKernelGGL(k_qr_update<T>, dim3((unsigned)h.size(), tiles), dim3(BS), 0, s, d_desc, j0,
                         (const double*)tbuf);
      SPAQR_HIP(hipGetLastError());
      ++*launches;
    }
  }
}

template <typename T>
void launch_trsm(const TrsmDesc* d_desc, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_trsm<T>, dim3(n), dim3(BS), 0, s, d_desc);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_owner(const OwnerDesc* d_desc, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_owner<T>, dim3(n), dim3(BS), 0, s, d_desc);
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
  template void launch_qr<T>(const QRDesc*, const std::vector<QRDesc>&, double*, hipStream_t,   \
                             int*);                                                            \
  template void launch_trsm<T>(const TrsmDesc*, int, hipStream_t);                             \
  template void launch_owner<T>(const OwnerDesc*, int, hipStream_t);                           \
  template void launch_rowcopy<T>(const RowCopyDesc*, int, int, hipStream_t);                         \
  template void launch_extract<T>(const ExtractDesc*, int, hipStream_t);                       \
  template void launch_scatter<T>(const ScatterDesc*, int, hipStream_t);

SPAQR_INST(double)
SPAQR_INST(float)

}  // namespace spaqr
