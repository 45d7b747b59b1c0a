// Vector kernels of preconditioned CGLS (Section 4) in FP64: reductions
// with a fixed summation order (per-block partials, then one block), and
// the fused updates of one iteration.  Scalars live in device memory so an
// iteration needs no host round trip.
#include <hip/hip_runtime.h>

#include "cgls.h"

namespace spaqr {

namespace {

constexpr int BS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// part[block] = sum_i (w_i v_i)^2 (w == nullptr: weights 1) or sum a_i b_i.
__global__ __launch_bounds__(BS) void k_dot_part(const double* __restrict__ a,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ w, int64_t n,
                                                 double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    double x = a[i];
    if (w) x *= w[i];
    acc += x * (b ? b[i] * (w ? w[i] : 1.0) : x);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(BS) void k_dot_final(const double* __restrict__ part, int np,
                                                  double* __restrict__ out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += BS) acc += part[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// y += alpha p (length n), r -= alpha q (length m), alpha = sc[G] / sc[QQ]
__global__ void k_step(double* __restrict__ y, const double* __restrict__ p, int64_t n,
                       double* __restrict__ r, const double* __restrict__ q, int64_t m,
                       const double* __restrict__ sc) {
  const double alpha = sc[SC_G] / sc[SC_QQ];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += alpha * p[i];
  if (i < m) r[i] -= alpha * q[i];
}

// p = s + (sc[GN] / sc[G]) p
__global__ void k_pupdate(double* __restrict__ p, const double* __restrict__ s, int64_t n,
                          const double* __restrict__ sc) {
  const double beta = sc[SC_GN] / sc[SC_G];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = s[i] + beta * p[i];
}

__global__ void k_set(double* __restrict__ sc, int dst, int src) { sc[dst] = sc[src]; }

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// d = s / w  (or s * w when mul)
__global__ void k_scale(double* __restrict__ d, const double* __restrict__ s,
                        const double* __restrict__ w, int64_t n, int mul) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = mul ? s[i] * w[i] : s[i] / w[i];
}

// d = a - s
__global__ void k_sub(double* __restrict__ d, const double* __restrict__ a,
                      const double* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = a[i] - s[i];
}

inline unsigned nb(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

}  // namespace

int dot_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + BS - 1) / BS)); }

void launch_dot(const double* a, const double* b, const double* w, int64_t n, double* part,
                double* out, hipStream_t s) {
  const int np = dot_blocks(n);
  hipLaunchKernelGGL(k_dot_part, dim3(np), dim3(BS), 0, s, a, b, w, n, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(BS), 0, s, (const double*)part, np, out);
  SPAQR_HIP(hipGetLastError());
}

void launch_step(double* y, const double* p, int64_t n, double* r, const double* q, int64_t m,
                 const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_step, dim3(nb(std::max(n, m))), dim3(BS), 0, s, y, p, n, r, q, m, sc);
  SPAQR_HIP(hipGetLastError());
}

void launch_pupdate(double* p, const double* sv, int64_t n, const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_pupdate, dim3(nb(n)), dim3(BS), 0, s, p, sv, n, sc);
  SPAQR_HIP(hipGetLastError());
}

void launch_set(double* sc, int dst, int src, hipStream_t s) {
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, s, sc, dst, src);
  SPAQR_HIP(hipGetLastError());
}

void launch_copy(double* d, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3(nb(n)), dim3(BS), 0, s, d, src, n);
  SPAQR_HIP(hipGetLastError());
}

void launch_scale(double* d, const double* src, const double* w, int64_t n, bool mul, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale, dim3(nb(n)), dim3(BS), 0, s, d, src, w, n, mul ? 1 : 0);
  SPAQR_HIP(hipGetLastError());
}

void launch_sub(double* d, const double* a, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sub, dim3(nb(n)), dim3(BS), 0, s, d, a, src, n);
  SPAQR_HIP(hipGetLastError());
}

}  // namespace spaqr
