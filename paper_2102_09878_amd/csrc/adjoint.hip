// Device kernels of the column scaling (Algorithm 1: every column of A is
// scaled to unit 2-norm before partitioning and factorization) and of the
// least-squares adjoint: the gradient of a loss of x*(A, b) with respect
// to b and to the stored nonzeros of A,
//   dL/db = A lambda,   dL/dA_ij = r_i lambda_j - (A lambda)_i x_j,
// with A^T A lambda = dL/dx and r = b - A x.
#include <hip/hip_runtime.h>

#include "cgls.h"

namespace spaqr {

namespace {

constexpr int BS = 256;

inline unsigned nb(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

// One thread per column j of A, walking column j through the transposed
// pattern (entries in ascending row order): D_j = ||A_{:,j}||_2, and the
// scaled value A_ij / D_j written to both the CSR and the transposed copy.
// bad[0] is set when a column has zero norm.
__global__ void k_colscale(const int64_t* __restrict__ at_ptr, const int64_t* __restrict__ at_src,
                           const double* __restrict__ vals, int64_t n, double* __restrict__ D,
                           double* __restrict__ ahat, double* __restrict__ ahatT, int* __restrict__ bad) {
  const int64_t j = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int64_t e = at_ptr[j]; e < at_ptr[j + 1]; ++e) {
    const double v = vals[at_src[e]];
    s += v * v;
  }
  if (!(s > 0.0)) {
    bad[0] = 1;
    D[j] = 1.0;
    return;
  }
  const double d = sqrt(s);
  D[j] = d;
  for (int64_t e = at_ptr[j]; e < at_ptr[j + 1]; ++e) {
    const int64_t k = at_src[e];
    const double v = vals[k] / d;
    ahatT[e] = v;
    ahat[k] = v;
  }
}

// One thread per row i: g[e] = r_i lam_j - al_i x_j for the entries e of row i.
__global__ void k_adj_grad(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ r, const double* __restrict__ al,
                           const double* __restrict__ lam, const double* __restrict__ x, int64_t m,
                           double* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= m) return;
  const double ri = r[i], ai = al[i];
  for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    const int j = col[e];
    g[e] = ri * lam[j] - ai * x[j];
  }
}

}  // namespace

void launch_colscale(const int64_t* at_ptr, const int64_t* at_src, const double* vals, int64_t n,
                     double* D, double* ahat, double* ahatT, int* bad, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_colscale, dim3(nb(n)), dim3(BS), 0, s, at_ptr, at_src, vals, n, D, ahat, ahatT, bad);
  SPAQR_HIP(hipGetLastError());
}

void launch_adj_grad(const int64_t* row_ptr, const int32_t* col, const double* r, const double* al,
                     const double* lam, const double* x, int64_t m, double* g, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_adj_grad, dim3(nb(m)), dim3(BS), 0, s, row_ptr, col, r, al, lam, x, m, g);
  SPAQR_HIP(hipGetLastError());
}

}  // namespace spaqr
