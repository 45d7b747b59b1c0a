// Solves with the spaQR factor: CGLS with right preconditioner D^-1 W^-1
// (Section 4), the one-shot seminormal solve (Section 1) and the adjoint
// solve A^T A lambda = g preconditioned by the same factor; plus the column
// scaling that precedes everything (Algorithm 1).  All vector work runs in
// device kernels; the host only reads one residual norm per iteration to
// decide whether to stop.
#include <chrono>
#include <cmath>
#include <cstring>

#include "cgls.h"
#include "handle.h"

namespace spaqr {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Vecs {
  double *y, *p, *u, *s, *t, *r, *q, *part, *sc;
};

Vecs workspace(Handle& H) {
  const size_t N = H.P.N, M = H.P.M;
  const size_t need = 5 * N + 2 * M + 1024 + SC_N;
  if (H.cg_elems < need) {
    if (H.d_cg) SPAQR_HIP(hipFree(H.d_cg));
    H.d_cg = nullptr;
    if (hipMalloc(&H.d_cg, need * sizeof(double)) != hipSuccess)
      throw Error(SPAQR_ENOMEM, "device allocation failed");
    H.cg_elems = need;
  }
  double* b = H.d_cg;
  Vecs v;
  v.y = b;
  v.p = b + N;
  v.u = b + 2 * N;
  v.s = b + 3 * N;
  v.t = b + 4 * N;
  v.r = b + 5 * N;
  v.q = b + 5 * N + M;
  v.part = b + 5 * N + 2 * M;
  v.sc = v.part + 1024;
  return v;
}

// t = Ahat^T r  (Ahat = A D^-1)
void atmul(Handle& H, const double* r, double* t) {
  launch_spmv(H.d_atp, H.d_ati, H.d_ahatT, r, t, H.P.N, H.stream);
}
// q = Ahat u
void amul(Handle& H, const double* u, double* q) {
  launch_spmv(H.d_rp, H.d_ci, H.d_ahat, u, q, H.P.M, H.stream);
}

double read_scalar(Handle& H, const double* d) {
  SPAQR_HIP(hipMemcpyAsync(H.h_sc, d, sizeof(double), hipMemcpyDeviceToHost, H.stream));
  SPAQR_HIP(hipStreamSynchronize(H.stream));
  return H.h_sc[0];
}

}  // namespace

void csne(Handle& H, const double* b, double* x) {
  if (!H.factored) throw Error(SPAQR_ESTATE, "factorize first");
  Vecs v = workspace(H);
  const int64_t N = H.P.N;
  atmul(H, b, v.t);
  apply_op(H, true, v.t);
  apply_op(H, false, v.t);
  launch_scale(x, v.t, H.d_D, N, false, H.stream);
  SPAQR_HIP(hipStreamSynchronize(H.stream));
  H.kt.harvest();
}

int cgls(Handle& H, const double* b, double tol, int max_iter, double* x, spaqr_cgls_info* info) {
  if (!H.factored) throw Error(SPAQR_ESTATE, "factorize first");
  if (!(tol >= 0.0) || max_iter < 0) throw Error(SPAQR_EARG, "bad tolerance or iteration limit");
  const double t0 = now_s();
  Vecs v = workspace(H);
  const int64_t N = H.P.N, M = H.P.M;
  hipStream_t st = H.stream;
  // r = b, t = Ahat^T r, ||A^T b|| = ||D t||
  launch_copy(v.r, b, M, st);
  atmul(H, v.r, v.t);
  launch_dot(v.t, nullptr, H.d_D, N, v.part, v.sc + SC_ATB, st);
  launch_dot(b, nullptr, nullptr, M, v.part, v.sc + SC_TRUE, st);
  // s = W^-T t, p = s, gamma = ||s||^2, y = 0
  launch_copy(v.s, v.t, N, st);
  apply_op(H, true, v.s);
  launch_copy(v.p, v.s, N, st);
  launch_dot(v.s, nullptr, nullptr, N, v.part, v.sc + SC_G, st);
  SPAQR_HIP(hipMemsetAsync(v.y, 0, N * sizeof(double), st));
  SPAQR_HIP(hipMemcpyAsync(H.h_sc, v.sc, SC_N * sizeof(double), hipMemcpyDeviceToHost, st));
  SPAQR_HIP(hipStreamSynchronize(st));
  const double atb = std::sqrt(H.h_sc[SC_ATB]);
  const double nb = std::sqrt(H.h_sc[SC_TRUE]);
  const double normA = H.normA;
  const double denom = normA * nb;
  double res = denom > 0 ? atb / denom : 0.0;
  int it = 0;
  while (res > tol && it < max_iter) {
    // q = Ahat W^-1 p
    launch_copy(v.u, v.p, N, st);
    apply_op(H, false, v.u);
    amul(H, v.u, v.q);
    launch_dot(v.q, nullptr, nullptr, M, v.part, v.sc + SC_QQ, st);
    launch_step(v.y, v.p, N, v.r, v.q, M, v.sc, st);
    // t = Ahat^T r, ||A^T r|| = ||D t||
    atmul(H, v.r, v.t);
    launch_dot(v.t, nullptr, H.d_D, N, v.part, v.sc + SC_TT, st);
    // s = W^-T t, p = s + beta p
    launch_copy(v.s, v.t, N, st);
    apply_op(H, true, v.s);
    launch_dot(v.s, nullptr, nullptr, N, v.part, v.sc + SC_GN, st);
    launch_pupdate(v.p, v.s, N, v.sc, st);
    launch_set(v.sc, SC_G, SC_GN, st);
    ++it;
    res = std::sqrt(read_scalar(H, v.sc + SC_TT)) / denom;
  }
  // x = D^-1 W^-1 y and the true residual in FP64
  launch_copy(v.u, v.y, N, st);
  apply_op(H, false, v.u);
  launch_scale(x, v.u, H.d_D, N, false, st);
  amul(H, v.u, v.q);
  launch_sub(v.r, b, v.q, M, st);
  atmul(H, v.r, v.t);
  launch_dot(v.t, nullptr, H.d_D, N, v.part, v.sc + SC_TT, st);
  const double tt = std::sqrt(read_scalar(H, v.sc + SC_TT));
  H.kt.harvest();
  const bool conv = res <= tol;
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->residual = denom > 0 ? tt / denom : 0.0;
    info->paper_residual = atb > 0 ? tt / atb : 0.0;
    info->norm_a = normA;
    info->seconds = now_s() - t0;
  }
  return conv ? SPAQR_OK : SPAQR_NOCONV;
}

void scale_values(Handle& H) {
  Vecs v = workspace(H);
  const int64_t N = H.P.N, M = H.P.M;
  hipStream_t st = H.stream;
  SPAQR_HIP(hipMemsetAsync(H.d_flag, 0, sizeof(int), st));
  launch_colscale(H.d_atp, H.d_atsrc, H.d_vals, N, H.d_D, H.d_ahat, H.d_ahatT, H.d_flag, st);
  SPAQR_HIP(hipMemcpyAsync(H.h_sc + 8, H.d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SPAQR_HIP(hipStreamSynchronize(st));
  int bad = 0;
  std::memcpy(&bad, H.h_sc + 8, sizeof(int));
  if (bad) throw Error(SPAQR_EARG, "a column of A has zero norm");
  // ||A||_2: 30 power steps on A^T A = D Ahat^T Ahat D from the all-ones
  // vector (a lower bound of the norm)
  launch_fill(v.p, 1.0 / std::sqrt((double)N), N, st);
  for (int it = 0; it < 30; ++it) {
    launch_scale(v.u, v.p, H.d_D, N, true, st);
    amul(H, v.u, v.q);
    atmul(H, v.q, v.t);
    launch_scale(v.t, v.t, H.d_D, N, true, st);
    launch_dot(v.t, nullptr, nullptr, N, v.part, v.sc + SC_PW, st);
    launch_normalize(v.p, v.t, N, v.sc, SC_PW, st);
  }
  const double lam2 = read_scalar(H, v.sc + SC_PW);
  H.normA = std::sqrt(std::sqrt(lam2));
  (void)M;
}

int adjoint(Handle& H, const double* x, const double* b, const double* g, double tol, int max_iter,
            double* grad_b, double* grad_vals, double* lambda, spaqr_cgls_info* info) {
  if (!H.factored) throw Error(SPAQR_ESTATE, "factorize first");
  if (!(tol >= 0.0) || max_iter < 0) throw Error(SPAQR_EARG, "bad tolerance or iteration limit");
  const double t0 = now_s();
  Vecs v = workspace(H);
  const int64_t N = H.P.N, M = H.P.M;
  hipStream_t st = H.stream;
  // In mu = D lambda:  (Ahat^T Ahat) mu = D^-1 g, preconditioned by W^-1 W^-T.
  // v.y = mu, v.t = residual, v.s = z, v.p = search direction.
  launch_scale(v.t, g, H.d_D, N, false, st);
  launch_dot(g, nullptr, nullptr, N, v.part, v.sc + SC_TRUE, st);
  launch_copy(v.s, v.t, N, st);
  apply_op(H, true, v.s);
  apply_op(H, false, v.s);
  launch_copy(v.p, v.s, N, st);
  launch_dot(v.t, v.s, nullptr, N, v.part, v.sc + SC_G, st);
  SPAQR_HIP(hipMemsetAsync(v.y, 0, N * sizeof(double), st));
  const double ng = std::sqrt(read_scalar(H, v.sc + SC_TRUE));
  double res = ng > 0 ? 1.0 : 0.0;
  int it = 0;
  while (res > tol && it < max_iter) {
    amul(H, v.p, v.q);
    atmul(H, v.q, v.u);
    launch_dot(v.p, v.u, nullptr, N, v.part, v.sc + SC_QQ, st);
    launch_step(v.y, v.p, N, v.t, v.u, N, v.sc, st);
    launch_dot(v.t, nullptr, H.d_D, N, v.part, v.sc + SC_TT, st);
    launch_copy(v.s, v.t, N, st);
    apply_op(H, true, v.s);
    apply_op(H, false, v.s);
    launch_dot(v.t, v.s, nullptr, N, v.part, v.sc + SC_GN, st);
    launch_pupdate(v.p, v.s, N, v.sc, st);
    launch_set(v.sc, SC_G, SC_GN, st);
    ++it;
    res = std::sqrt(read_scalar(H, v.sc + SC_TT)) / ng;
  }
  // lambda = D^-1 mu (into v.s), A lambda = Ahat mu (into v.q)
  launch_scale(v.s, v.y, H.d_D, N, false, st);
  if (lambda) launch_copy(lambda, v.s, N, st);
  amul(H, v.y, v.q);
  if (grad_b) launch_copy(grad_b, v.q, M, st);
  // true residual g - A^T A lambda = g - D Ahat^T (A lambda)
  atmul(H, v.q, v.u);
  launch_scale(v.u, v.u, H.d_D, N, true, st);
  launch_sub(v.u, g, v.u, N, st);
  launch_dot(v.u, nullptr, nullptr, N, v.part, v.sc + SC_TT, st);
  // r = b - A x = b - Ahat (D x)
  if (grad_vals) {
    launch_scale(v.t, x, H.d_D, N, true, st);
    amul(H, v.t, v.r);
    launch_sub(v.r, b, v.r, M, st);
    launch_adj_grad(H.d_rp, H.d_ci, v.r, v.q, v.s, x, M, grad_vals, st);
  }
  const double tr = std::sqrt(read_scalar(H, v.sc + SC_TT));
  H.kt.harvest();
  const bool conv = res <= tol;
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->residual = ng > 0 ? tr / ng : 0.0;
    info->paper_residual = res;
    info->norm_a = H.normA;
    info->seconds = now_s() - t0;
  }
  return conv ? SPAQR_OK : SPAQR_NOCONV;
}

}  // namespace spaqr
