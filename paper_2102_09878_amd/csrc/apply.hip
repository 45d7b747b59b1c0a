// Device kernels that apply the spaQR factor and run CGLS (gfx950, wave64).
//
// W is a product of elementary ops (Section 2.7): eliminations
// [R_ss R_sN; 0 I], scalings R_pp and sparsifications Q_pp = H_1..H_r.
// W^-1 is applied op by op from the last to the first, W^-T from the first
// to the last with transposes.  Ops created in one round never write a slot
// another op of the round reads, so a round is one batched launch (one
// block per op); only the neighbour updates x_N -= R_sN^T x_s of W^-T can
// meet on a shared neighbour, and they go through a staging buffer summed
// per slot in op order, which keeps every application bit-reproducible.
// Factors may be FP32; every accumulation is FP64, so the preconditioner
// stays a fixed linear operator for CGLS.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "spaqr_impl.h"
#include "wave.h"

namespace spaqr {

namespace {

constexpr int BS = 256;
constexpr int UPW = 32;  // row-update loads in flight per thread
constexpr int APPLY_MAX = 4096;  // largest cluster handled by one block (32 KB LDS vector)

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum63(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Solve R t = t (upper, column-major, ld) in place in LDS, blocks of 64:
// the block's diagonal 64 x 64 tile is staged in LDS by all threads (one
// round trip), wave 0 solves it without barriers or memory waits, then all
// threads update the rows above it.
template <typename T>
__device__ void trsv_upper(const T* __restrict__ R, int64_t ld, int n, double* t, T (*Ds)[65]) {
  const int tid = threadIdx.x, lane = tid & 63;
  for (int jb = ((n - 1) / 64) * 64; jb >= 0; jb -= 64) {
    const int nb = min(n, jb + 64) - jb;
    for (int e = tid; e < 64 * 64; e += BS) {
      const int r = e & 63, c = e >> 6;
      if (r < nb && c < nb) Ds[c][r] = R[jb + r + (int64_t)(jb + c) * ld];
    }
    __syncthreads();
    if (tid < 64) {
      double v = lane < nb ? t[jb + lane] : 0.0;
      for (int c = nb - 1; c >= 0; --c) {
        if (lane == c) v = v / (double)Ds[c][c];
        const double tj = lane_bcast(v, c);
        if (lane < c) v -= tj * (double)Ds[c][lane];
      }
      if (lane < nb) t[jb + lane] = v;
    }
    __syncthreads();
    // rows above the block: loads issued 32 at a time ahead of the (ordered) sums
    const int ldi = (int)ld;
    for (int i = tid; i < jb; i += BS) {
      const T* rp = R + (int64_t)jb * ld + i;
      double acc = 0.0;
#pragma unroll 1
      for (int h = 0; h < 64; h += UPW) {
        T rv[UPW];
#pragma unroll
        for (int c = 0; c < UPW; ++c) rv[c] = rp[min(h + c, nb - 1) * ldi];
#pragma unroll
        for (int c = 0; c < UPW; ++c)
          if (h + c < nb) acc += (double)rv[c] * t[jb + h + c];
      }
      t[i] -= acc;
    }
    __syncthreads();
  }
}

// Solve R^T y = t (R upper) in place, forward over blocks of 64 (diagonal
// tile staged in LDS as above).
template <typename T>
__device__ void trsv_upper_t(const T* __restrict__ R, int64_t ld, int n, double* t, T (*Ds)[65]) {
  const int tid = threadIdx.x, lane = tid & 63;
  for (int jb = 0; jb < n; jb += 64) {
    const int je = min(n, jb + 64), nb = je - jb;
    for (int e = tid; e < 64 * 64; e += BS) {
      const int r = e & 63, c = e >> 6;
      if (r < nb && c < nb) Ds[c][r] = R[jb + r + (int64_t)(jb + c) * ld];
    }
    __syncthreads();
    if (tid < 64) {
      double v = lane < nb ? t[jb + lane] : 0.0;
      for (int c = 0; c < nb; ++c) {
        if (lane == c) v = v / (double)Ds[c][c];
        const double yj = lane_bcast(v, c);
        if (lane > c && lane < nb) v -= (double)Ds[lane][c] * yj;
      }
      if (lane < nb) t[jb + lane] = v;
    }
    __syncthreads();
    for (int k = je + tid; k < n; k += BS) {
      const T* col = R + (int64_t)k * ld + jb;
      double acc = 0.0;
#pragma unroll 1
      for (int h = 0; h < 64; h += UPW) {
        T rv[UPW];
#pragma unroll
        for (int c = 0; c < UPW; ++c) rv[c] = col[min(h + c, nb - 1)];
#pragma unroll
        for (int c = 0; c < UPW; ++c)
          if (h + c < nb) acc += (double)rv[c] * t[jb + h + c];
      }
      t[k] -= acc;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_apply(const ApplyOp* __restrict__ ops, int transpose,
                                              double* __restrict__ x, double* __restrict__ work) {
  const ApplyOp op = ops[blockIdx.x];
  __shared__ double t[APPLY_MAX];
  __shared__ double sh[4];
  __shared__ T Ds[64][65];  // diagonal tile of the triangular solves
  const int tid = threadIdx.x;
  const int n1 = op.n1;
  const T* R = static_cast<const T*>(op.R);
  if (n1 <= 0) return;  // uniform over the block
  for (int i = tid; i < n1; i += BS) t[i] = x[op.s1[i]];
  __syncthreads();
  if (op.kind == 0) {  // eliminate
    const double* pw = work + op.poff;
    if (!transpose) {
      // t = x_s - R_sN x_N from the chunk partials (summed in chunk order)
      if (op.n2 > 0)
        for (int i = tid; i < n1; i += BS) {
          double a = 0.0;
          for (int k = 0; k < op.nchunk; ++k) a += pw[(int64_t)k * n1 + i];
          t[i] -= a;
        }
      __syncthreads();
      trsv_upper(R, op.ld, n1, t, Ds);
      for (int i = tid; i < n1; i += BS) x[op.s1[i]] = t[i];
    } else {
      trsv_upper_t(R, op.ld, n1, t, Ds);
      for (int i = tid; i < n1; i += BS) {
        x[op.s1[i]] = t[i];
        if (op.n2 > 0) work[op.poff + i] = t[i];
      }
    }
  } else if (op.kind == 1) {  // scale
    if (!transpose)
      trsv_upper(R, op.ld, n1, t, Ds);
    else
      trsv_upper_t(R, op.ld, n1, t, Ds);
    for (int i = tid; i < n1; i += BS) x[op.s1[i]] = t[i];
  } else {  // sparsify: Q = H_0 .. H_{r-1}
    const int r = op.n2;
    const T* tau = static_cast<const T*>(op.tau);
    if (n1 <= 256) {
      // one wave: a lane owns entries lane, lane + 64, ..., so the
      // reflectors need no barrier, only a wave reduction each
      if (tid < 64) {
        // lane l takes rows k + l + 64 j of reflector k; the next reflector's
        // entries (and tau) are loaded while the current one is applied
        T vn[4];
        T taun = T(0);
        auto fetch = [&](int s, T (&v4)[4], T& tk) {
          const int k = transpose ? s : r - 1 - s;
          const T* v = R + (int64_t)k * op.ld;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int i = k + tid + 64 * j;
            v4[j] = i < n1 ? v[i] : T(0);
          }
          tk = tau[k];
        };
        if (r > 0) fetch(0, vn, taun);
        for (int s = 0; s < r; ++s) {
          const int k = transpose ? s : r - 1 - s;
          T vc[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) vc[j] = vn[j];
          const T tk = taun;
          if (s + 1 < r) fetch(s + 1, vn, taun);
          double part = 0.0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int i = k + tid + 64 * j;
            if (i < n1) part += (double)vc[j] * t[i];
          }
          const double f = (double)tk * wave_sum(part);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int i = k + tid + 64 * j;
            if (i < n1) t[i] -= f * (double)vc[j];
          }
        }
      }
      __syncthreads();
    } else {
      for (int s = 0; s < r; ++s) {
        const int k = transpose ? s : r - 1 - s;
        const T* v = R + (int64_t)k * op.ld;
        double part = 0.0;
        for (int i = k + tid; i < n1; i += BS) part += (double)v[i] * t[i];
        const double dot = block_sum(part, sh);
        const double f = (double)tau[k] * dot;
        for (int i = k + tid; i < n1; i += BS) t[i] -= f * (double)v[i];
        __syncthreads();
      }
    }
    for (int i = tid; i < n1; i += BS) x[op.s1[i]] = t[i];
  }
}

// One (op, chunk) of the neighbour products, columns [c0, c0 + APPLY_CHUNK).
// W^-1: work[poff + k n1 + i] = sum_c R_sN[i, c] x[s2[c]]; the chunk's x
// values are staged in LDS and rows are spread over the threads (when n1 is
// small the threads also split the columns, summed in a fixed order).
// W^-T: stage[nstage + c] = sum_i R_sN[i, c] t_i with t from work[poff ..];
// each wave takes four columns at a time, lanes over rows (coalesced).
template <typename T>
__global__ __launch_bounds__(BS) void k_apply_gemv(const ApplyOp* __restrict__ ops, const int2* __restrict__ chunks,
                                                   int transpose, const double* __restrict__ x,
                                                   double* __restrict__ stage, double* __restrict__ work) {
  const int2 ck = chunks[blockIdx.x];
  const ApplyOp op = ops[ck.x];
  const int n1 = op.n1;
  const int c0 = ck.y * APPLY_CHUNK, c1 = min(op.n2, c0 + APPLY_CHUNK);
  const T* RN = static_cast<const T*>(op.R) + (int64_t)n1 * op.ld;
  const int tid = threadIdx.x;
  __shared__ double v[APPLY_MAX > APPLY_CHUNK ? APPLY_MAX : APPLY_CHUNK];
  if (!transpose) {
    for (int c = c0 + tid; c < c1; c += BS) v[c - c0] = x[op.s2[c]];
    __syncthreads();
    double* out = work + op.poff + (int64_t)ck.y * n1;
    const int rows = (n1 + 63) / 64 * 64;
    const int ns = rows >= BS ? 1 : BS / rows;  // column slices
    const int sl = tid / rows, i0 = tid % rows;
    __shared__ double part[BS];
    for (int ib = 0; ib < n1; ib += (rows >= BS ? BS : rows)) {
      const int i = ib + (rows >= BS ? tid : i0);
      double acc = 0.0;
      if (sl < ns && i < n1) {
        // 16 columns' loads issued ahead of their sums (columns in the same order)
        const T* ri = RN + i;
#pragma unroll 1
        for (int c = c0 + sl; c < c1; c += 16 * ns) {
          T rv[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) rv[u] = ri[(int64_t)min(c + u * ns, c1 - 1) * op.ld];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (c + u * ns < c1) acc += (double)rv[u] * v[c + u * ns - c0];
        }
      }
      if (ns == 1) {
        if (sl == 0 && i < n1) out[i] = acc;
      } else {
        part[tid] = acc;
        __syncthreads();
        if (sl == 0 && i < n1) {
          double a = 0.0;
          for (int k = 0; k < ns; ++k) a += part[k * rows + i0];
          out[i] = a;
        }
        __syncthreads();
      }
    }
  } else {
    for (int i = tid; i < n1; i += BS) v[i] = work[op.poff + i];
    __syncthreads();
    const int wv = tid >> 6, lane = tid & 63;
    for (int cb = c0 + 4 * wv; cb < c1; cb += 16) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      const T* col = RN + (int64_t)cb * op.ld;
      const int nc = min(4, c1 - cb);
      for (int i = lane; i < n1; i += 64) {
        const double ti = v[i];
        a0 += (double)col[i] * ti;
        if (nc > 1) a1 += (double)col[i + op.ld] * ti;
        if (nc > 2) a2 += (double)col[i + 2 * op.ld] * ti;
        if (nc > 3) a3 += (double)col[i + 3 * op.ld] * ti;
      }
      a0 = wave_sum63(a0);
      a1 = wave_sum63(a1);
      a2 = wave_sum63(a2);
      a3 = wave_sum63(a3);
      if (lane == 63) {
        double* out = stage + op.nstage + cb;
        out[0] = a0;
        if (nc > 1) out[1] = a1;
        if (nc > 2) out[2] = a2;
        if (nc > 3) out[3] = a3;
      }
    }
  }
}

// x[nslots[k]] -= sum of stage[noff[e]] for e in [nptr[k], nptr[k+1]), in order
__global__ void k_apply_nsum(const int* __restrict__ nslots, const int* __restrict__ nptr,
                             const int* __restrict__ noff, int n, const double* __restrict__ stage,
                             double* __restrict__ x) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double acc = 0.0;
  for (int e = nptr[k]; e < nptr[k + 1]; ++e) acc += stage[noff[e]];
  x[nslots[k]] -= acc;
}

__global__ void k_spmv(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                       const double* __restrict__ val, const double* __restrict__ x,
                       double* __restrict__ y, int64_t rows) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double acc = 0.0;
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) acc += val[e] * x[idx[e]];
  y[r] = acc;
}

}  // namespace

template <typename T>
void launch_apply_batch(const ApplyOp* d_ops, int n, int max_n1, bool transpose, double* x,
                        double* stage, double* work, hipStream_t s) {
  if (n <= 0) return;
  if (max_n1 > APPLY_MAX) throw Error(SPAQR_EARG, "cluster too large for the apply kernel");
  (void)stage;
  hipLaunchKernelGGL(k_apply<T>, dim3(n), dim3(BS), 0, s, d_ops, transpose ? 1 : 0, x, work);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
void launch_apply_gemv(const ApplyOp* d_ops, const int2* chunks, int nchunks, bool transpose, const double* x,
                       double* stage, double* work, hipStream_t s) {
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(k_apply_gemv<T>, dim3(nchunks), dim3(BS), 0, s, d_ops, chunks, transpose ? 1 : 0, x, stage,
                     work);
  SPAQR_HIP(hipGetLastError());
}

void launch_apply_nsum(const int* nslots, const int* nptr, const int* noff, int n, const double* stage,
                       double* x, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_apply_nsum, dim3((n + BS - 1) / BS), dim3(BS), 0, s, nslots, nptr, noff, n, stage, x);
  SPAQR_HIP(hipGetLastError());
}

void launch_spmv(const int64_t* ptr, const int32_t* idx, const double* val, const double* x,
                 double* y, int64_t rows, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_spmv, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, ptr, idx, val, x, y,
                     rows);
  SPAQR_HIP(hipGetLastError());
}

template void launch_apply_batch<double>(const ApplyOp*, int, int, bool, double*, double*, double*, hipStream_t);
template void launch_apply_batch<float>(const ApplyOp*, int, int, bool, double*, double*, double*, hipStream_t);
template void launch_apply_gemv<double>(const ApplyOp*, const int2*, int, bool, const double*, double*, double*,
                                        hipStream_t);
template void launch_apply_gemv<float>(const ApplyOp*, const int2*, int, bool, const double*, double*, double*,
                                       hipStream_t);

}  // namespace spaqr
