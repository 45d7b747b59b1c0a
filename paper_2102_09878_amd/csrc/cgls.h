// Launchers of the CGLS vector kernels (cgls.hip).
#pragma once

#include "spaqr_impl.h"

namespace spaqr {

// device scalar slots
enum { SC_G = 0, SC_QQ = 1, SC_TT = 2, SC_GN = 3, SC_ATB = 4, SC_TRUE = 5, SC_PW = 6, SC_N = 8 };

int dot_blocks(int64_t n);
// *out = sum_i a_i b_i (b == nullptr: sum a_i^2); with weights w: a_i w_i and b_i w_i.
void launch_dot(const double* a, const double* b, const double* w, int64_t n, double* part,
                double* out, hipStream_t s);
void launch_step(double* y, const double* p, int64_t n, double* r, const double* q, int64_t m,
                 const double* sc, hipStream_t s);
void launch_pupdate(double* p, const double* sv, int64_t n, const double* sc, hipStream_t s);
void launch_set(double* sc, int dst, int src, hipStream_t s);
void launch_copy(double* d, const double* src, int64_t n, hipStream_t s);
void launch_scale(double* d, const double* src, const double* w, int64_t n, bool mul, hipStream_t s);
void launch_sub(double* d, const double* a, const double* src, int64_t n, hipStream_t s);

// adjoint.hip
void launch_colscale(const int64_t* at_ptr, const int64_t* at_src, const double* vals, int64_t n,
                     double* D, double* ahat, double* ahatT, int* bad, hipStream_t s);
void launch_fill(double* d, double v, int64_t n, hipStream_t s);
void launch_normalize(double* d, const double* src, int64_t n, const double* sc, int slot, hipStream_t s);
void launch_adj_grad(const int64_t* row_ptr, const int32_t* col, const double* r, const double* al,
                     const double* lam, const double* x, int64_t m, double* g, hipStream_t s);

}  // namespace spaqr
