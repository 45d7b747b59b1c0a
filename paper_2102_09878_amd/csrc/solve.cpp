// Solves with the spaQR factor: CGLS with right preconditioner D^-1 W^-1
// (Section 4), the one-shot seminormal solve (Section 1) and the adjoint
// solve A^T A lambda = g preconditioned by the same factor; plus the column
// scaling that precedes everything (Algorithm 1).  All vector work runs in
// device kernels; the host reads one vector of residual norms per
// iteration to decide which problems go on.
//
// A plan may hold a batch of independent problems (block-diagonal union):
// products with A and the W sweeps act on all of them in one launch each,
// while every scalar of the recurrences and every stopping test is per
// problem.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
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
  const size_t N = H.P.N, M = H.P.M, G = H.P.count;
  const size_t need = 5 * N + 2 * M + G * SDOT_MAX_BLOCKS + G * SC_N;
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
  v.sc = v.part + G * SDOT_MAX_BLOCKS;
  return v;
}

int64_t longest(const std::vector<int64_t>& seg) {
  int64_t m = 0;
  for (size_t g = 0; g + 1 < seg.size(); ++g) m = std::max(m, seg[g + 1] - seg[g]);
  return m;
}
Segs cols(Handle& H) { return Segs{H.d_segc, H.P.count, longest(H.P.seg_col)}; }
Segs rows(Handle& H) { return Segs{H.d_segr, H.P.count, longest(H.P.seg_row)}; }

// t = Ahat^T r  (Ahat = A D^-1)
void atmul(Handle& H, const double* r, double* t) {
  launch_spmv(H.d_atp, H.d_ati, H.d_ahatT, r, t, H.P.N, H.stream);
}
// q = Ahat u
void amul(Handle& H, const double* u, double* q) {
  launch_spmv(H.d_rp, H.d_ci, H.d_ahat, u, q, H.P.M, H.stream);
}

// one slot of every problem's scalars, to the host
void read_slot(Handle& H, const double* sc, int slot, std::vector<double>& out) {
  const int G = H.P.count;
  SPAQR_HIP(hipMemcpyAsync(H.h_sc, sc, (size_t)G * SC_N * sizeof(double), hipMemcpyDeviceToHost, H.stream));
  SPAQR_HIP(hipStreamSynchronize(H.stream));
  out.resize(G);
  for (int g = 0; g < G; ++g) out[g] = H.h_sc[(size_t)g * SC_N + slot];
}

void upload_act(Handle& H, const std::vector<int>& act) {
  std::memcpy(H.h_act, act.data(), act.size() * sizeof(int));
  SPAQR_HIP(hipMemcpyAsync(H.d_act, H.h_act, act.size() * sizeof(int), hipMemcpyHostToDevice, H.stream));
}

}  // namespace

void scale_values(Handle& H) {
  Vecs v = workspace(H);
  const int64_t N = H.P.N;
  hipStream_t st = H.stream;
  SPAQR_HIP(hipMemsetAsync(H.d_flag, 0, sizeof(int), st));
  launch_colscale(H.d_atp, H.d_atsrc, H.d_vals, N, H.d_D, H.d_ahat, H.d_ahatT, H.d_flag, st);
  int bad = 0;
  SPAQR_HIP(hipMemcpyAsync(H.h_act, H.d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  SPAQR_HIP(hipStreamSynchronize(st));
  bad = H.h_act[0];
  if (bad) throw Error(SPAQR_EARG, "a column of A has zero norm");
  // ||A_g||_2: 30 power steps on A^T A = D Ahat^T Ahat D from the all-ones
  // vector of each problem (a lower bound of the norm)
  const Segs sc = cols(H);
  for (int g = 0; g < H.P.count; ++g) {
    const int64_t lo = H.P.seg_col[g], hi = H.P.seg_col[g + 1];
    launch_fill(v.p + lo, 1.0 / std::sqrt((double)(hi - lo)), hi - lo, st);
  }
  for (int it = 0; it < 30; ++it) {
    launch_scale(v.u, v.p, H.d_D, N, true, st);
    amul(H, v.u, v.q);
    atmul(H, v.q, v.t);
    launch_scale(v.t, v.t, H.d_D, N, true, st);
    launch_sdot(v.t, nullptr, nullptr, sc, v.part, v.sc, SC_PW, st);
    launch_normalize(v.p, v.t, sc, v.sc, SC_PW, st);
  }
  std::vector<double> lam2;
  read_slot(H, v.sc, SC_PW, lam2);
  H.normA.assign(H.P.count, 0.0);
  for (int g = 0; g < H.P.count; ++g) H.normA[g] = std::sqrt(std::sqrt(lam2[g]));
}

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

// Corrected seminormal equations with iterative refinement (Section 1).
// In scaled variables y = D x (A x = Ahat y, A^T A ~ D W^T W D):
//   y_0 = W^-1 W^-T Ahat^T b,  y_{k+1} = y_k + W^-1 W^-T Ahat^T (b - Ahat y_k),
// stopping once ||A^T r|| = ||D Ahat^T r|| <= tol ||A||_2 ||b|| for every
// problem of the plan (tested before each correction) or after max_steps
// corrections; x = D^-1 y.  infos[g] gets the corrections taken (iters)
// and problem g's final residuals.
int csne_refine(Handle& H, const double* b, double tol, int max_steps, double* x, spaqr_cgls_info* infos) {
  if (!H.factored) throw Error(SPAQR_ESTATE, "factorize first");
  if (!(tol >= 0.0) || max_steps < 0) throw Error(SPAQR_EARG, "bad tolerance or step limit");
  const double t0 = now_s();
  Vecs v = workspace(H);
  const int64_t N = H.P.N, M = H.P.M;
  const int G = H.P.count;
  const Segs sc = cols(H), sr = rows(H);
  hipStream_t st = H.stream;
  // ||A^T b|| and ||b|| per problem
  atmul(H, b, v.t);
  launch_sdot(v.t, nullptr, H.d_D, sc, v.part, v.sc, SC_ATB, st);
  launch_sdot(b, nullptr, nullptr, sr, v.part, v.sc, SC_TRUE, st);
  // y = W^-1 W^-T Ahat^T b
  launch_copy(v.y, v.t, N, st);
  apply_op(H, true, v.y);
  apply_op(H, false, v.y);
  std::vector<double> atb2, b2, tt;
  read_slot(H, v.sc, SC_ATB, atb2);
  for (int g = 0; g < G; ++g) b2.push_back(H.h_sc[(size_t)g * SC_N + SC_TRUE]);
  std::vector<double> denom(G), res(G);
  for (int g = 0; g < G; ++g) denom[g] = H.normA[g] * std::sqrt(b2[g]);
  int steps = 0;
  for (;;) {
    // r = b - Ahat y, t = Ahat^T r, ||A^T r|| = ||D t||
    amul(H, v.y, v.q);
    launch_sub(v.r, b, v.q, M, st);
    atmul(H, v.r, v.t);
    launch_sdot(v.t, nullptr, H.d_D, sc, v.part, v.sc, SC_TT, st);
    read_slot(H, v.sc, SC_TT, tt);
    bool all = true;
    for (int g = 0; g < G; ++g) {
      res[g] = denom[g] > 0 ? std::sqrt(tt[g]) / denom[g] : 0.0;
      all = all && res[g] <= tol;
    }
    if (all || steps >= max_steps) break;
    // y += W^-1 W^-T t
    apply_op(H, true, v.t);
    apply_op(H, false, v.t);
    launch_add(v.y, v.y, v.t, N, st);
    ++steps;
  }
  launch_scale(x, v.y, H.d_D, N, false, st);
  SPAQR_HIP(hipStreamSynchronize(st));
  H.kt.harvest();
  const double secs = now_s() - t0;
  bool conv = true;
  for (int g = 0; g < G; ++g) {
    conv = conv && res[g] <= tol;
    if (infos) {
      spaqr_cgls_info& info = infos[g];
      info.iters = steps;
      info.converged = res[g] <= tol ? 1 : 0;
      info.residual = res[g];
      const double atb = std::sqrt(atb2[g]);
      info.paper_residual = atb > 0 ? res[g] * denom[g] / atb : 0.0;
      info.norm_a = H.normA[g];
      info.seconds = secs;
    }
  }
  return conv ? SPAQR_OK : SPAQR_NOCONV;
}

int cgls(Handle& H, const double* b, double tol, int max_iter, double* x, spaqr_cgls_info* infos) {
  if (!H.factored) throw Error(SPAQR_ESTATE, "factorize first");
  if (!(tol >= 0.0) || max_iter < 0) throw Error(SPAQR_EARG, "bad tolerance or iteration limit");
  const double t0 = now_s();
  Vecs v = workspace(H);
  const int64_t N = H.P.N, M = H.P.M;
  const int G = H.P.count;
  const Segs sc = cols(H), sr = rows(H);
  hipStream_t st = H.stream;
  // r = b, t = Ahat^T r, ||A^T b|| = ||D t||
  launch_copy(v.r, b, M, st);
  atmul(H, v.r, v.t);
  launch_sdot(v.t, nullptr, H.d_D, sc, v.part, v.sc, SC_ATB, st);
  launch_sdot(b, nullptr, nullptr, sr, v.part, v.sc, SC_TRUE, st);
  // s = W^-T t, p = s, gamma = ||s||^2, y = 0
  launch_copy(v.s, v.t, N, st);
  apply_op(H, true, v.s);
  launch_copy(v.p, v.s, N, st);
  launch_sdot(v.s, nullptr, nullptr, sc, v.part, v.sc, SC_G, st);
  SPAQR_HIP(hipMemsetAsync(v.y, 0, N * sizeof(double), st));
  std::vector<double> atb2, b2;
  read_slot(H, v.sc, SC_ATB, atb2);
  for (int g = 0; g < G; ++g) b2.push_back(H.h_sc[(size_t)g * SC_N + SC_TRUE]);
  std::vector<double> denom(G), res(G), atb(G);
  std::vector<int> act(G), iters(G, 0);
  int nact = 0;
  for (int g = 0; g < G; ++g) {
    atb[g] = std::sqrt(atb2[g]);
    denom[g] = H.normA[g] * std::sqrt(b2[g]);
    res[g] = denom[g] > 0 ? atb[g] / denom[g] : 0.0;
    act[g] = res[g] > tol ? 1 : 0;
    nact += act[g];
  }
  upload_act(H, act);
  int it = 0;
  std::vector<double> tt;
  // one iteration's kernels (every argument a handle-owned pointer, so the
  // sequence can be recorded once and replayed)
  auto iteration = [&](hipStream_t ks) {
    // q = Ahat W^-1 p
    launch_copy(v.u, v.p, N, ks);
    apply_op_on(H, false, v.u, ks);
    launch_spmv(H.d_rp, H.d_ci, H.d_ahat, v.u, v.q, H.P.M, ks);
    launch_sdot(v.q, nullptr, nullptr, sr, v.part, v.sc, SC_QQ, ks);
    launch_step(v.y, v.p, sc, v.r, v.q, sr, H.d_act, v.sc, ks);
    // t = Ahat^T r, ||A^T r|| = ||D t||
    launch_spmv(H.d_atp, H.d_ati, H.d_ahatT, v.r, v.t, H.P.N, ks);
    launch_sdot(v.t, nullptr, H.d_D, sc, v.part, v.sc, SC_TT, ks);
    // s = W^-T t, p = s + beta p
    launch_copy(v.s, v.t, N, ks);
    apply_op_on(H, true, v.s, ks);
    launch_sdot(v.s, nullptr, nullptr, sc, v.part, v.sc, SC_GN, ks);
    launch_pupdate(v.p, v.s, sc, H.d_act, v.sc, ks);
    launch_set(v.sc, SC_G, SC_GN, H.d_act, G, ks);
  };
  // CGLS iterations replay one captured HIP graph (SPAQR_NO_GRAPH=1 keeps
  // the eager launches, which run the same kernels in the same order)
  const bool no_graph = std::getenv("SPAQR_NO_GRAPH") != nullptr;
  const bool graph = !no_graph && !H.kt.on("apply") && nact > 0 && max_iter > 0;
  if (graph && (!H.cg_exec || H.cg_key != H.apply_key || H.cg_base != H.d_cg)) {
    H.drop_cg_graph();
    if (!H.cap_stream) SPAQR_HIP(hipStreamCreateWithFlags(&H.cap_stream, hipStreamNonBlocking));
    SPAQR_HIP(hipStreamBeginCapture(H.cap_stream, hipStreamCaptureModeRelaxed));
    iteration(H.cap_stream);
    SPAQR_HIP(hipStreamEndCapture(H.cap_stream, &H.cg_graph));
    SPAQR_HIP(hipGraphInstantiate(&H.cg_exec, H.cg_graph, nullptr, nullptr, 0));
    H.cg_key = H.apply_key;
    H.cg_base = H.d_cg;
  }
  while (nact > 0 && it < max_iter) {
    if (graph)
      SPAQR_HIP(hipGraphLaunch(H.cg_exec, st));
    else
      iteration(st);
    ++it;
    read_slot(H, v.sc, SC_TT, tt);
    nact = 0;
    for (int g = 0; g < G; ++g) {
      if (!act[g]) continue;
      ++iters[g];
      res[g] = std::sqrt(tt[g]) / denom[g];
      act[g] = res[g] > tol ? 1 : 0;
      nact += act[g];
    }
    if (nact > 0) upload_act(H, act);
  }
  // x = D^-1 W^-1 y and the true residuals in FP64
  launch_copy(v.u, v.y, N, st);
  apply_op(H, false, v.u);
  launch_scale(x, v.u, H.d_D, N, false, st);
  amul(H, v.u, v.q);
  launch_sub(v.r, b, v.q, M, st);
  atmul(H, v.r, v.t);
  launch_sdot(v.t, nullptr, H.d_D, sc, v.part, v.sc, SC_TT, st);
  read_slot(H, v.sc, SC_TT, tt);
  std::fill(act.begin(), act.end(), 1);
  upload_act(H, act);
  SPAQR_HIP(hipStreamSynchronize(st));  // h_act is reused by the next call
  H.kt.harvest();
  const double secs = now_s() - t0;
  bool all = true;
  for (int g = 0; g < G; ++g) {
    const bool conv = res[g] <= tol;
    all = all && conv;
    if (infos) {
      spaqr_cgls_info& info = infos[g];
      const double trn = std::sqrt(tt[g]);
      info.iters = iters[g];
      info.converged = conv ? 1 : 0;
      info.residual = denom[g] > 0 ? trn / denom[g] : 0.0;
      info.paper_residual = atb[g] > 0 ? trn / atb[g] : 0.0;
      info.norm_a = H.normA[g];
      info.seconds = secs;
    }
  }
  return all ? SPAQR_OK : SPAQR_NOCONV;
}

int adjoint(Handle& H, const double* x, const double* b, const double* g, double tol, int max_iter,
            double* grad_b, double* grad_vals, double* lambda, spaqr_cgls_info* info) {
  if (!H.factored) throw Error(SPAQR_ESTATE, "factorize first");
  if (H.P.count != 1) throw Error(SPAQR_EARG, "the adjoint solve takes a single-problem handle");
  if (!(tol >= 0.0) || max_iter < 0) throw Error(SPAQR_EARG, "bad tolerance or iteration limit");
  const double t0 = now_s();
  Vecs v = workspace(H);
  const int64_t N = H.P.N, M = H.P.M;
  const Segs sc = cols(H);
  hipStream_t st = H.stream;
  // In mu = D lambda:  (Ahat^T Ahat) mu = D^-1 g, preconditioned by W^-1 W^-T.
  // v.y = mu, v.t = residual, v.s = z, v.p = search direction.
  launch_scale(v.t, g, H.d_D, N, false, st);
  launch_sdot(g, nullptr, nullptr, sc, v.part, v.sc, SC_TRUE, st);
  launch_copy(v.s, v.t, N, st);
  apply_op(H, true, v.s);
  apply_op(H, false, v.s);
  launch_copy(v.p, v.s, N, st);
  launch_sdot(v.t, v.s, nullptr, sc, v.part, v.sc, SC_G, st);
  SPAQR_HIP(hipMemsetAsync(v.y, 0, N * sizeof(double), st));
  std::vector<double> tmp;
  read_slot(H, v.sc, SC_TRUE, tmp);
  const double ng = std::sqrt(tmp[0]);
  double res = ng > 0 ? 1.0 : 0.0;
  int it = 0;
  while (res > tol && it < max_iter) {
    amul(H, v.p, v.q);
    atmul(H, v.q, v.u);
    launch_sdot(v.p, v.u, nullptr, sc, v.part, v.sc, SC_QQ, st);
    launch_step(v.y, v.p, sc, v.t, v.u, sc, nullptr, v.sc, st);
    launch_sdot(v.t, nullptr, H.d_D, sc, v.part, v.sc, SC_TT, st);
    launch_copy(v.s, v.t, N, st);
    apply_op(H, true, v.s);
    apply_op(H, false, v.s);
    launch_sdot(v.t, v.s, nullptr, sc, v.part, v.sc, SC_GN, st);
    launch_pupdate(v.p, v.s, sc, nullptr, v.sc, st);
    launch_set(v.sc, SC_G, SC_GN, nullptr, 1, st);
    ++it;
    read_slot(H, v.sc, SC_TT, tmp);
    res = std::sqrt(tmp[0]) / ng;
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
  launch_sdot(v.u, nullptr, nullptr, sc, v.part, v.sc, SC_TT, st);
  // r = b - A x = b - Ahat (D x)
  if (grad_vals) {
    launch_scale(v.t, x, H.d_D, N, true, st);
    amul(H, v.t, v.r);
    launch_sub(v.r, b, v.r, M, st);
    launch_adj_grad(H.d_rp, H.d_ci, v.r, v.q, v.s, x, M, grad_vals, st);
  }
  read_slot(H, v.sc, SC_TT, tmp);
  const double tr = std::sqrt(tmp[0]);
  H.kt.harvest();
  const bool conv = res <= tol;
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->residual = ng > 0 ? tr / ng : 0.0;
    info->paper_residual = res;
    info->norm_a = H.normA[0];
    info->seconds = now_s() - t0;
  }
  return conv ? SPAQR_OK : SPAQR_NOCONV;
}

}  // namespace spaqr
