// Vector kernels of preconditioned CGLS (Section 4) and of the adjoint CG,
// in FP64.  Reductions have a fixed summation order (per-block partials,
// then one block per problem), so every solve is bit-reproducible; the
// scalars stay in device memory, so an iteration needs one host read only
// (the residual norms that decide when to stop).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cgls.h"
#include "wave.h"

namespace spaqr {

namespace {

constexpr int BS = 256;

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

__device__ __forceinline__ bool frozen(const int* act, int g) { return act && !act[g]; }

// part[g * nblk + bx] = partial sum over segment g (grid: nblk x count)
__global__ __launch_bounds__(BS) void k_sdot_part(const double* __restrict__ a, const double* __restrict__ b,
                                                  const double* __restrict__ w, const int64_t* __restrict__ seg,
                                                  int nblk, double* __restrict__ part) {
  __shared__ double sh[4];
  const int g = blockIdx.y;
  const int64_t lo = seg[g], hi = seg[g + 1];
  double acc = 0.0;
  for (int64_t i = lo + (int64_t)blockIdx.x * BS + threadIdx.x; i < hi; i += (int64_t)nblk * BS) {
    double x = a[i];
    if (w) x *= w[i];
    acc += x * (b ? b[i] * (w ? w[i] : 1.0) : x);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)g * nblk + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// sc[g * SC_N + slot] = sum of the nblk partials of segment g (grid: count)
__global__ __launch_bounds__(BS) void k_sdot_final(const double* __restrict__ part, int nblk,
                                                   double* __restrict__ sc, int slot) {
  __shared__ double sh[4];
  const int g = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += BS) acc += part[(int64_t)g * nblk + i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sc[g * SC_N + slot] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_step(double* __restrict__ y, const double* __restrict__ p, const int64_t* __restrict__ sy,
                       double* __restrict__ r, const double* __restrict__ q, const int64_t* __restrict__ sr,
                       const int* __restrict__ act, const double* __restrict__ sc) {
  const int g = blockIdx.y;
  if (frozen(act, g)) return;
  const double alpha = sc[g * SC_N + SC_G] / sc[g * SC_N + SC_QQ];
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (sy[g] + i < sy[g + 1]) y[sy[g] + i] += alpha * p[sy[g] + i];
  if (sr[g] + i < sr[g + 1]) r[sr[g] + i] -= alpha * q[sr[g] + i];
}

__global__ void k_pupdate(double* __restrict__ p, const double* __restrict__ s, const int64_t* __restrict__ seg,
                          const int* __restrict__ act, const double* __restrict__ sc) {
  const int g = blockIdx.y;
  if (frozen(act, g)) return;
  const double beta = sc[g * SC_N + SC_GN] / sc[g * SC_N + SC_G];
  const int64_t i = seg[g] + (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < seg[g + 1]) p[i] = s[i] + beta * p[i];
}

__global__ void k_set(double* __restrict__ sc, int dst, int src, const int* __restrict__ act, int count) {
  const int g = blockIdx.x * BS + threadIdx.x;
  if (g < count && !frozen(act, g)) sc[g * SC_N + dst] = sc[g * SC_N + src];
}

__global__ void k_normalize(double* __restrict__ d, const double* __restrict__ s, const int64_t* __restrict__ seg,
                            const double* __restrict__ sc, int slot) {
  const int g = blockIdx.y;
  const double f = 1.0 / sqrt(sc[g * SC_N + slot]);
  const int64_t i = seg[g] + (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < seg[g + 1]) d[i] = s[i] * f;
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// d = s / w  (or s * w when mul)
__global__ void k_scale(double* __restrict__ d, const double* __restrict__ s, const double* __restrict__ w,
                        int64_t n, int mul) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) d[i] = mul ? s[i] * w[i] : s[i] / w[i];
}

// d = a - s
__global__ void k_sub(double* __restrict__ d, const double* __restrict__ a, const double* __restrict__ s,
                      int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) d[i] = a[i] - s[i];
}

__global__ void k_add(double* __restrict__ d, const double* __restrict__ a, const double* __restrict__ s,
                      int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) d[i] = a[i] + s[i];
}

__global__ void k_fill(double* __restrict__ d, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) d[i] = v;
}

inline unsigned nb(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + BS - 1) / BS); }

}  // namespace

void launch_sdot(const double* a, const double* b, const double* w, const Segs& sg, double* part, double* sc,
                 int slot, hipStream_t s) {
  if (sg.count <= 0) return;
  const int nblk = (int)std::min<int64_t>(SDOT_MAX_BLOCKS, std::max<int64_t>(1, (sg.max_len + 2 * BS - 1) / (2 * BS)));
  hipLaunchKernelGGL(k_sdot_part, dim3(nblk, sg.count), dim3(BS), 0, s, a, b, w, sg.seg, nblk, part);
  hipLaunchKernelGGL(k_sdot_final, dim3(sg.count), dim3(BS), 0, s, (const double*)part, nblk, sc, slot);
  SPAQR_HIP(hipGetLastError());
}

void launch_step(double* y, const double* p, const Segs& sy, double* r, const double* q, const Segs& sr,
                 const int* act, const double* sc, hipStream_t s) {
  if (sy.count <= 0) return;
  hipLaunchKernelGGL(k_step, dim3(nb(std::max(sy.max_len, sr.max_len)), sy.count), dim3(BS), 0, s, y, p, sy.seg,
                     r, q, sr.seg, act, sc);
  SPAQR_HIP(hipGetLastError());
}

void launch_pupdate(double* p, const double* sv, const Segs& sg, const int* act, const double* sc, hipStream_t s) {
  if (sg.count <= 0) return;
  hipLaunchKernelGGL(k_pupdate, dim3(nb(sg.max_len), sg.count), dim3(BS), 0, s, p, sv, sg.seg, act, sc);
  SPAQR_HIP(hipGetLastError());
}

void launch_set(double* sc, int dst, int src, const int* act, int count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_set, dim3(nb(count)), dim3(BS), 0, s, sc, dst, src, act, count);
  SPAQR_HIP(hipGetLastError());
}

void launch_normalize(double* d, const double* src, const Segs& sg, const double* sc, int slot, hipStream_t s) {
  if (sg.count <= 0) return;
  hipLaunchKernelGGL(k_normalize, dim3(nb(sg.max_len), sg.count), dim3(BS), 0, s, d, src, sg.seg, sc, slot);
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

void launch_add(double* d, const double* a, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_add, dim3(nb(n)), dim3(BS), 0, s, d, a, src, n);
  SPAQR_HIP(hipGetLastError());
}

void launch_fill(double* d, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nb(n)), dim3(BS), 0, s, d, v, n);
  SPAQR_HIP(hipGetLastError());
}

}  // namespace spaqr
