// Launchers of the solver vector kernels (cgls.hip, adjoint.hip).
//
// Vectors may hold several independent problems back to back (a batch):
// problem g owns elements [seg[g], seg[g+1]).  Reductions and scalar
// updates are per problem; the scalars of problem g live at
// sc[g * SC_N + slot] in device memory, and act[g] == 0 (act non-null)
// freezes problem g.
#pragma once

#include "spaqr_impl.h"

namespace spaqr {

enum { SC_G = 0, SC_QQ = 1, SC_TT = 2, SC_GN = 3, SC_ATB = 4, SC_TRUE = 5, SC_PW = 6, SC_N = 8 };
constexpr int SDOT_MAX_BLOCKS = 512;  // partial sums per problem

struct Segs {
  const int64_t* seg;  // count + 1 offsets (device)
  int count;
  int64_t max_len;     // longest segment
};

// sc[g, slot] = sum over segment g of a_i b_i (b == nullptr: a_i^2); with
// weights w the terms are (a_i w_i)(b_i w_i).  part: count * SDOT_MAX_BLOCKS.
void launch_sdot(const double* a, const double* b, const double* w, const Segs& sg, double* part,
                 double* sc, int slot, hipStream_t s);
// y += alpha_g p over segments sy, r -= alpha_g q over segments sr,
// alpha_g = sc[g, G] / sc[g, QQ]
void launch_step(double* y, const double* p, const Segs& sy, double* r, const double* q, const Segs& sr,
                 const int* act, const double* sc, hipStream_t s);
// p = s + (sc[g, GN] / sc[g, G]) p
void launch_pupdate(double* p, const double* sv, const Segs& sg, const int* act, const double* sc,
                    hipStream_t s);
// sc[g, dst] = sc[g, src]
void launch_set(double* sc, int dst, int src, const int* act, int count, hipStream_t s);
// d = src / sqrt(sc[g, slot])
void launch_normalize(double* d, const double* src, const Segs& sg, const double* sc, int slot, hipStream_t s);

void launch_copy(double* d, const double* src, int64_t n, hipStream_t s);
void launch_scale(double* d, const double* src, const double* w, int64_t n, bool mul, hipStream_t s);
void launch_sub(double* d, const double* a, const double* src, int64_t n, hipStream_t s);
void launch_add(double* d, const double* a, const double* src, int64_t n, hipStream_t s);
void launch_fill(double* d, double v, int64_t n, hipStream_t s);

// adjoint.hip
void launch_colscale(const int64_t* at_ptr, const int64_t* at_src, const double* vals, int64_t n,
                     double* D, double* ahat, double* ahatT, int* bad, hipStream_t s);
void launch_adj_grad(const int64_t* row_ptr, const int32_t* col, const double* r, const double* al,
                     const double* lam, const double* x, int64_t m, double* g, hipStream_t s);

}  // namespace spaqr
