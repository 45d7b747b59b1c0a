// Batched blocked Householder QR for gfx950 (wave64): the block Householder
// eliminations of Section 2.3 and the interface scalings of Section 2.4.
//
// Reflectors follow the LAPACK convention (beta = -sign(alpha)||x||,
// sign(0) = +1, tau = 0 for a zero tail) and are applied left to right, so
// every front sees exactly the reflector sequence of an unblocked
// column-by-column Householder QR; blocking only regroups the updates.
//
// Panel (QR_NB columns):
//  * one work-group per front when fronts are short (the leaf level: many
//    fronts of ~1000 rows in one launch);
//  * row-split over QR_RS-row segments when a front is tall (fronts of
//    10^4 rows that are eliminated alone): per column, one launch applies
//    the previous reflector to the segment and forms norm partials, one
//    launch forms the reflector and the dot partials for the remaining
//    panel columns.  Partials are reduced in a fixed order (deterministic).
// Trailing update C <- (I - V T V^T)^T C over (front, 64-column tile, row
// segment) blocks: W_s = V_s^T C_s per segment, W = T^T sum_s W_s, then
// C_s -= V_s W.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "handle.h"
#include "spaqr_impl.h"
#include "wave.h"

namespace spaqr {

namespace {

constexpr int BS = 256;
constexpr int NB = QR_NB;
constexpr int TN = QR_TN;
constexpr int RS = QR_RS;

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum63(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 63) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Reflector scalars in LAPACK's convention (beta = -sign(alpha) ||x||,
// sign(0) = +1), where an alpha of at most SIGN_FLOOR u ||x|| (u the FP64
// unit roundoff, whatever the storage type) counts as 0: it is a structural
// zero carrying rounding error, whose sign two evaluations may not agree
// on.  (FP32 rounding can exceed that floor; there the FP32 form may flip
// an R row relative to the FP64 form: an equivalent factor.)
constexpr double SIGN_FLOOR = 64.0 * 1.1102230246251565e-16;
__device__ __forceinline__ void house_scalars(double alpha, double xn2, double& beta, double& tau,
                                              double& scal) {
  if (xn2 == 0.0) {
    beta = alpha;
    tau = 0.0;
    scal = 1.0;
  } else {
    const double nrm = sqrt(alpha * alpha + xn2);
    const double s = (alpha < 0.0 && -alpha > SIGN_FLOOR * nrm) ? -1.0 : 1.0;
    beta = -s * nrm;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
}

// T of the compact-WY form (upper triangular, kb x kb, stored NB x NB
// row-major at Tg) from tau and the strictly-upper Gram G[a][b] = v_a^T v_b:
// T[i][i] = tau_i, T[a][i] = -tau_i sum_{b=a}^{i-1} T[a][b] G[b][i].  Built
// in LDS column by column (threads over rows a), then written out.  All
// threads of the block must call it.
__device__ void build_t(double* __restrict__ Tg, const double* s_tau, const double (*G)[NB + 1], int kb,
                        double (*Ts)[NB + 1]) {
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += BS) Ts[e / NB][e % NB] = 0.0;
  __syncthreads();
  for (int i = 0; i < kb; ++i) {
    if (tid < i) {
      double acc = 0.0;
      for (int b = tid; b < i; ++b) acc += Ts[tid][b] * G[b][i];
      Ts[tid][i] = -s_tau[i] * acc;
    } else if (tid == i) {
      Ts[i][i] = s_tau[i];
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += BS) Tg[e] = Ts[e / NB][e % NB];
}

// Partial Gram of the panel's reflectors over rows [r0, r1): out[a][b] for
// a < b < kb of sum_r v_a[r] v_b[r], where v_a has 1 at row j0+a, zeros
// above and the stored reflector below.  64-row tiles of V go through LDS;
// thread t accumulates entries (t / 8, 4 (t % 8) .. + 3).  All threads of
// the block must call it.
template <typename T>
__device__ void gram_rows(const T* __restrict__ A, int64_t lda, int j0, int kb, int r0, int r1,
                          double (*Vs)[NB + 1], double* acc4) {
  const int tid = threadIdx.x;
  const int a = tid >> 3, b0 = (tid & 7) * 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) acc4[k] = 0.0;
  for (int rb = r0; rb < r1; rb += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * NB; e += BS) {
      const int rr = e & 63, c = e >> 6;
      const int r = rb + rr;
      double v = 0.0;
      if (r < r1 && c < kb) {
        const int rc = j0 + c;
        v = r == rc ? 1.0 : (r > rc ? (double)A[r + (int64_t)rc * lda] : 0.0);
      }
      Vs[rr][c] = v;
    }
    __syncthreads();
    const int nr = min(64, r1 - rb);
    for (int rr = 0; rr < nr; ++rr) {
      const double va = Vs[rr][a];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc4[k] += va * Vs[rr][b0 + k];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int seg_lo(int j0) { return j0 / RS; }
__device__ __forceinline__ int seg_hi(int m) { return (m + RS - 1) / RS; }

// ---------------------------------------------------------------------------
// panel, one work-group per front
// ---------------------------------------------------------------------------
// Each thread owns the rows j0 + tid + k BS of the panel for the whole
// panel, so a column step needs no data exchange besides the block
// reductions: (a) ||tail||^2 and alpha -> reflector scalars, (b) scale the
// owned part of v_i, (c) one accumulation pass over the owned rows forming
// the kb-1 dot products v_i^T y_j (j > i, trailing panel columns) and
// v_a^T v_i (a < i, Gram column of T) together, (d) update the owned rows
// and extend T by one column in LDS.
template <typename T>
__global__ __launch_bounds__(BS) void k_qr_panel(const QRDesc* __restrict__ D, int j0,
                                                 double* __restrict__ tbuf) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  T* A = static_cast<T*>(d.A);
  T* tau = static_cast<T*>(d.tau);
  const int64_t lda = d.lda;
  const int m = d.m;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  __shared__ double sh[4];
  __shared__ double red[4][NB];
  __shared__ double sv[NB];
  __shared__ double gcol[NB];
  __shared__ double fj[NB];
  __shared__ double Ts[NB][NB + 1];

  for (int e = tid; e < NB * NB; e += BS) Ts[e / NB][e % NB] = 0.0;
  for (int i = 0; i < kb; ++i) {
    const int c = j0 + i;
    T* col = A + (int64_t)c * lda;
    // (a)
    double part = 0.0;
    for (int r = j0 + tid; r < m; r += BS)
      if (r > c) {
        const double v = col[r];
        part += v * v;
      }
    const double xn2 = block_sum(part, sh);
    const double alpha = col[c];
    double beta, tv, scal;
    house_scalars(alpha, xn2, beta, tv, scal);
    const double tvT = (double)static_cast<T>(tv);
    // (b)
    if (tv != 0.0)
      for (int r = j0 + tid; r < m; r += BS)
        if (r > c) col[r] = static_cast<T>(col[r] * scal);
    // (c) value q: a = q for q < i (Gram), column j = q + 1 for q >= i (dots)
    double acc[NB - 1];
#pragma unroll
    for (int q = 0; q < NB - 1; ++q) acc[q] = 0.0;
    for (int r = j0 + tid; r < m; r += BS) {
      if (r <= c) continue;
      const double vi = col[r];
#pragma unroll
      for (int q = 0; q < NB - 1; ++q)
        if (q < kb - 1) acc[q] += vi * (double)A[r + (int64_t)(j0 + (q < i ? q : q + 1)) * lda];
    }
#pragma unroll
    for (int q = 0; q < NB - 1; ++q) {
      if (q < kb - 1) {
        const double w = wave_sum63(acc[q]);
        if (lane == 63) red[wv][q] = w;
      }
    }
    __syncthreads();
    if (tid < kb - 1) sv[tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    __syncthreads();
    // (d)
    if (tid < kb - 1) {
      if (tid < i) {
        gcol[tid] = sv[tid] + (double)A[c + (int64_t)(j0 + tid) * lda];
      } else {
        const T* y = A + (int64_t)(j0 + tid + 1) * lda;
        fj[tid + 1] = tv * (sv[tid] + (double)y[c]);
      }
    }
    __syncthreads();
    if (tid < i) {
      double a2 = 0.0;
      for (int b2 = tid; b2 < i; ++b2) a2 += Ts[tid][b2] * gcol[b2];
      Ts[tid][i] = -tvT * a2;
    } else if (tid == i) {
      Ts[i][i] = tvT;
    }
    if (tv != 0.0) {
      for (int r = j0 + tid; r < m; r += BS) {
        if (r <= c) continue;
        const double vi = col[r];
        for (int j = i + 1; j < kb; ++j) {
          T* y = A + (int64_t)(j0 + j) * lda + r;
          *y = static_cast<T>((double)*y - fj[j] * vi);
        }
      }
      if (tid >= i && tid < kb - 1) {
        T* y = A + (int64_t)(j0 + tid + 1) * lda + c;
        *y = static_cast<T>((double)*y - fj[tid + 1]);
      }
    }
    __syncthreads();
    if (tid == 0) {
      col[c] = static_cast<T>(beta);
      tau[c] = static_cast<T>(tv);
    }
    __syncthreads();
  }
  double* Tg = tbuf + (int64_t)blockIdx.x * NB * NB;
  for (int e = tid; e < NB * NB; e += BS) Tg[e] = Ts[e / NB][e % NB];
}

// Same column steps with the panel held in registers (FP32 fronts of at
// most 2048 rows below j0): 512 threads, thread t owning rows j0 + t + 512 k
// (k < 4) of all NB panel columns.  The owner of row c = j0 + i publishes
// that row to LDS at the start of step i; everything else stays in
// registers until the panel is written back once at the end.
constexpr int PBS = 512;
constexpr int PRPT = 4;

// One column step of the register panel; I is a compile-time column so all
// register indexing is static.
template <int I>
__device__ __forceinline__ void panel_step(float (&P)[PRPT][NB], int j0, int m, int kb, float* tau,
                                           double* sh, double (*red)[NB], double* sv, double* gcol, double* fj,
                                           double* rowc, double (*Ts)[NB + 1]) {
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int c = j0 + I;
  const int oc = I % PBS, kc = I / PBS;
  // one pass over the rows below c: ||x||^2 and x^T A[c+1:, q] for the other
  // panel columns (x = A[c+1:, c], not yet scaled), reduced together; a
  // thread sums its (at most PRPT) rows in FP32, the reduction is FP64
  double part = 0.0;
  float acc[NB - 1];
#pragma unroll
  for (int q = 0; q < NB - 1; ++q) acc[q] = 0.0f;
#pragma unroll
  for (int k = 0; k < PRPT; ++k) {
    const int r = j0 + tid + PBS * k;
    if (tid == oc && k == kc)
#pragma unroll
      for (int q = 0; q < NB; ++q) rowc[q] = P[k][q];
    if (r <= c || r >= m) continue;
    const float xi = P[k][I];
    part += (double)xi * (double)xi;
#pragma unroll
    for (int q = 0; q < NB - 1; ++q) acc[q] = fmaf(xi, P[k][q < I ? q : q + 1], acc[q]);
  }
#pragma unroll
  for (int q = 0; q < NB - 1; ++q) {
    if (q < kb - 1) {
      const double w = wave_sum63((double)acc[q]);
      if (lane == 63) red[wv][q] = w;
    }
  }
  part = wave_sum63(part);
  if (lane == 63) red[wv][NB - 1] = part;
  __syncthreads();
  if (tid < kb - 1 || tid == NB - 1)
    sv[tid] = ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) +
              ((red[4][tid] + red[5][tid]) + (red[6][tid] + red[7][tid]));
  __syncthreads();
  const double xn2 = sv[NB - 1];
  const double alpha = rowc[I];
  double beta, tv, scal;
  house_scalars(alpha, xn2, beta, tv, scal);
  const double tvT = (double)static_cast<float>(tv);
  if (tid < kb - 1) {
    const double svq = tv != 0.0 ? scal * sv[tid] : sv[tid];
    if (tid < I)
      gcol[tid] = svq + rowc[tid];
    else
      fj[tid + 1] = tv * (svq + rowc[tid + 1]);
  }
  __syncthreads();
  if (tid < I) {
    double a2 = 0.0;
    for (int b2 = tid; b2 < I; ++b2) a2 += Ts[tid][b2] * gcol[b2];
    Ts[tid][I] = -tvT * a2;
  } else if (tid == I) {
    Ts[I][I] = tvT;
  }
#pragma unroll
  for (int k = 0; k < PRPT; ++k) {
    const int r = j0 + tid + PBS * k;
    if (r < c || r >= m) continue;
    if (r == c) {
#pragma unroll
      for (int q = I + 1; q < NB; ++q)
        if (q < kb && tv != 0.0) P[k][q] = static_cast<float>((double)P[k][q] - fj[q]);
      P[k][I] = static_cast<float>(beta);
    } else if (tv != 0.0) {
      P[k][I] = static_cast<float>(P[k][I] * scal);
      const double vi = P[k][I];
#pragma unroll
      for (int q = I + 1; q < NB; ++q)
        if (q < kb) P[k][q] = static_cast<float>((double)P[k][q] - fj[q] * vi);
    }
  }
  if (tid == 0) tau[c] = static_cast<float>(tv);
  __syncthreads();
}

template <int I>
__device__ __forceinline__ void panel_steps(float (&P)[PRPT][NB], int j0, int m, int kb, float* tau, double* sh,
                                            double (*red)[NB], double* sv, double* gcol, double* fj, double* rowc,
                                            double (*Ts)[NB + 1]) {
  if constexpr (I < NB) {
    if (I >= kb) return;
    panel_step<I>(P, j0, m, kb, tau, sh, red, sv, gcol, fj, rowc, Ts);
    panel_steps<I + 1>(P, j0, m, kb, tau, sh, red, sv, gcol, fj, rowc, Ts);
  }
}

__global__ __launch_bounds__(PBS) void k_qr_panel_reg(const QRDesc* __restrict__ D, int j0,
                                                      double* __restrict__ tbuf) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  float* A = static_cast<float*>(d.A);
  float* tau = static_cast<float*>(d.tau);
  const int64_t lda = d.lda;
  const int m = d.m;
  const int tid = threadIdx.x;
  __shared__ double sh[8];
  __shared__ double red[8][NB];
  __shared__ double sv[NB];
  __shared__ double gcol[NB];
  __shared__ double fj[NB];
  __shared__ double rowc[NB];
  __shared__ double Ts[NB][NB + 1];

  float P[PRPT][NB];
#pragma unroll
  for (int k = 0; k < PRPT; ++k) {
    const int r = j0 + tid + PBS * k;
#pragma unroll
    for (int q = 0; q < NB; ++q) P[k][q] = (r < m && q < kb) ? A[r + (int64_t)(j0 + q) * lda] : 0.0f;
  }
  for (int e = tid; e < NB * NB; e += PBS) Ts[e / NB][e % NB] = 0.0;
  __syncthreads();
  panel_steps<0>(P, j0, m, kb, tau, sh, red, sv, gcol, fj, rowc, Ts);
#pragma unroll
  for (int k = 0; k < PRPT; ++k) {
    const int r = j0 + tid + PBS * k;
    if (r < m)
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < kb) A[r + (int64_t)(j0 + q) * lda] = P[k][q];
  }
  double* Tg = tbuf + (int64_t)blockIdx.x * NB * NB;
  for (int e = tid; e < NB * NB; e += PBS) Tg[e] = Ts[e / NB][e % NB];
}

// ---------------------------------------------------------------------------
// panel of tall fronts, one cooperative launch per panel
//
// Work-group (f, s) holds rows j0 + s TSEG .. + TSEG of front f in registers
// (PR rows per thread: 4 in FP32, the ownership of the register panel above;
// 2 in FP64, so a thread holds the same 128 registers of panel values).  Each column step needs two
// sums over all row segments of the front - ||tail||^2 and the kb-1 dot
// products - exchanged through small global buffers across two grid
// barriers.  The step loop runs to the largest panel width of the launch in
// every work-group, so all of them reach every barrier.
// ---------------------------------------------------------------------------
template <typename T>
struct CoopRows {
  static constexpr int PR = sizeof(T) == 4 ? PRPT : PRPT / 2;
  static constexpr int TSEG = PBS * PR;
};

struct CoopShared {
  double sh[8];
  double red[8][NB];
  double sv[NB];
  double gcol[NB];
  double fj[NB];
  double rowc[NB];
  double Ts[NB][NB + 1];
};

template <typename T, int PR, int I>
__device__ __forceinline__ void coop_step(T (&P)[PR][NB], int j0, int m, int kb, int rbase, int sg, int S,
                                          T* tau, double* dpb, double* rowc_g, CoopShared& L) {
  namespace cg = cooperative_groups;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const bool work = I < kb;
  const int c = j0 + I;
  double* rowc_i = rowc_g + (I & 1) * NB;
  // Column I's partials, double-buffered by column parity: slots 0 .. NB-2
  // hold x^T A[c+1:, q] of the other panel columns (x = A[c+1:, c], not yet
  // scaled), slot NB-1 holds ||x||^2, so one grid barrier serves both sums.
  // (A buffer is rewritten two columns later, after every work-group has
  // passed the barrier in between and so has read it.)
  double* dp = dpb + (I & 1) * S * NB;
  if (work) {
    double part = 0.0;
    T acc[NB - 1];
#pragma unroll
    for (int q = 0; q < NB - 1; ++q) acc[q] = T(0);
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      const int r = rbase + tid + PBS * k;
      if (r <= c || r >= m) continue;
      const T xi = P[k][I];
      part += (double)xi * (double)xi;
#pragma unroll
      for (int q = 0; q < NB - 1; ++q) acc[q] = fma(xi, P[k][q < I ? q : q + 1], acc[q]);
    }
    // row c lives in segment 0, thread I, slot 0
    if (sg == 0 && tid == I)
#pragma unroll
      for (int q = 0; q < NB; ++q) rowc_i[q] = P[0][q];
#pragma unroll
    for (int q = 0; q < NB - 1; ++q) {
      const double w = wave_sum63((double)acc[q]);
      if (lane == 63) L.red[wv][q] = w;
    }
    part = wave_sum63(part);
    if (lane == 63) L.red[wv][NB - 1] = part;
    __syncthreads();
    if (tid < kb - 1 || tid == NB - 1)
      dp[sg * NB + tid] = ((L.red[0][tid] + L.red[1][tid]) + (L.red[2][tid] + L.red[3][tid])) +
                          ((L.red[4][tid] + L.red[5][tid]) + (L.red[6][tid] + L.red[7][tid]));
  }
  cg::this_grid().sync();
  // reflector scalars (identical in every segment), sums over the segments,
  // T column, update of the owned rows
  if (work) {
    double xn2 = 0.0;
    for (int t = 0; t < S; ++t) xn2 += dp[t * NB + NB - 1];
    if (tid < NB) L.rowc[tid] = rowc_i[tid];
    __syncthreads();
    double beta, tv, scal;
    house_scalars(L.rowc[I], xn2, beta, tv, scal);
    const double tvT = (double)static_cast<T>(tv);
    if (tid < kb - 1) {
      double a = 0.0;
      for (int t = 0; t < S; ++t) a += dp[t * NB + tid];
      const double sv = tv != 0.0 ? scal * a : a;
      if (tid < I)
        L.gcol[tid] = sv + L.rowc[tid];
      else
        L.fj[tid + 1] = tv * (sv + L.rowc[tid + 1]);
    }
    __syncthreads();
    if (tid < I) {
      double a2 = 0.0;
      for (int b2 = tid; b2 < I; ++b2) a2 += L.Ts[tid][b2] * L.gcol[b2];
      L.Ts[tid][I] = -tvT * a2;
    } else if (tid == I) {
      L.Ts[I][I] = tvT;
    }
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      const int r = rbase + tid + PBS * k;
      if (r < c || r >= m) continue;
      if (r == c) {
#pragma unroll
        for (int q = I + 1; q < NB; ++q)
          if (q < kb && tv != 0.0) P[k][q] = static_cast<T>((double)P[k][q] - L.fj[q]);
        P[k][I] = static_cast<T>(beta);
      } else if (tv != 0.0) {
        P[k][I] = static_cast<T>(P[k][I] * scal);
        const double vi = P[k][I];
#pragma unroll
        for (int q = I + 1; q < NB; ++q)
          if (q < kb) P[k][q] = static_cast<T>((double)P[k][q] - L.fj[q] * vi);
      }
    }
    if (sg == 0 && tid == 0) tau[c] = static_cast<T>(tv);
  }
  __syncthreads();
}

// kbmax is the same in every work-group, so every one runs the same steps
// and reaches every grid barrier.
template <typename T, int PR, int I>
__device__ __forceinline__ void coop_steps(T (&P)[PR][NB], int j0, int m, int kb, int kbmax, int rbase, int sg,
                                           int S, T* tau, double* dp, double* rowc_g, CoopShared& L) {
  if constexpr (I < NB) {
    if (I >= kbmax) return;
    coop_step<T, PR, I>(P, j0, m, kb, rbase, sg, S, tau, dp, rowc_g, L);
    coop_steps<T, PR, I + 1>(P, j0, m, kb, kbmax, rbase, sg, S, tau, dp, rowc_g, L);
  }
}

template <typename T>
__global__ __launch_bounds__(PBS) void k_qrp_coop(const QRDesc* __restrict__ D, int j0, int kbmax, int S,
                                                  QRWork ws) {
  constexpr int PR = CoopRows<T>::PR;
  const int f = blockIdx.x / S, sg = blockIdx.x % S;
  const QRDesc d = D[f];
  const int kk = min(d.m, d.k);
  const int kb = j0 < kk ? min(NB, kk - j0) : 0;
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int m = d.m;
  const int tid = threadIdx.x;
  const int rbase = j0 + sg * CoopRows<T>::TSEG;
  __shared__ CoopShared L;
  T P[PR][NB];
#pragma unroll
  for (int k = 0; k < PR; ++k) {
    const int r = rbase + tid + PBS * k;
#pragma unroll
    for (int q = 0; q < NB; ++q) P[k][q] = (r < m && q < kb) ? A[r + (int64_t)(j0 + q) * lda] : T(0);
  }
  for (int e = tid; e < NB * NB; e += PBS) L.Ts[e / NB][e % NB] = 0.0;
  __syncthreads();
  coop_steps<T, PR, 0>(P, j0, m, kb, kbmax, rbase, sg, S, static_cast<T*>(d.tau),
                       ws.dp + (int64_t)f * 2 * ws.MS * NB, ws.gp + (int64_t)f * ws.MS * NB * NB, L);
#pragma unroll
  for (int k = 0; k < PR; ++k) {
    const int r = rbase + tid + PBS * k;
    if (r < m)
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < kb) A[r + (int64_t)(j0 + q) * lda] = P[k][q];
  }
  if (sg == 0 && kb > 0) {
    double* Tg = ws.tbuf + (int64_t)f * NB * NB;
    for (int e = tid; e < NB * NB; e += PBS) Tg[e] = L.Ts[e / NB][e % NB];
  }
}

// ---------------------------------------------------------------------------
// panel, row-split (tall fronts)
// ---------------------------------------------------------------------------

// Step a(i): apply reflector i-1 to the segment's rows of panel columns
// j0+i .. j0+kb-1 (dots reduced from step b(i-1)), finalise column j0+i-1,
// then publish the segment's partial ||A[j0+i+1:, j0+i]||^2.
template <typename T>
__global__ __launch_bounds__(BS) void k_qrp_a(const QRDesc* __restrict__ D, int j0, int i, QRWork ws) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  if (i > kb) return;
  const int f = blockIdx.x, s = blockIdx.y;
  const int m = d.m;
  const int r0 = max(j0, s * RS), r1 = min(m, (s + 1) * RS);
  if (r0 >= r1) return;
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int tid = threadIdx.x;
  const int c = j0 + i;
  __shared__ double sh[4];
  __shared__ double w[NB];
  if (i > 0) {
    const int pc = c - 1;
    const int ncol = j0 + kb - c;
    if (tid < ncol) {
      double acc = 0.0;
      for (int sg = seg_lo(j0); sg < seg_hi(m); ++sg) acc += ws.dp[((int64_t)f * ws.MS + sg) * NB + (c - j0) + tid];
      w[tid] = acc;
    }
    __syncthreads();
    const double tp = (double)static_cast<const T*>(d.tau)[pc];
    if (tp != 0.0) {
      const T* vcol = A + (int64_t)pc * lda;
      for (int r = max(r0, pc) + tid; r < r1; r += BS) {
        const double v = r == pc ? 1.0 : (double)vcol[r];
        for (int j = 0; j < ncol; ++j) {
          T* y = A + (int64_t)(c + j) * lda + r;
          *y = static_cast<T>((double)*y - tp * w[j] * v);
        }
      }
    }
    if (tid == 0 && pc >= r0 && pc < r1) A[pc + (int64_t)pc * lda] = static_cast<T>(ws.betas[f]);
  }
  if (i < kb) {
    // same thread-to-row mapping as the update above: no barrier needed
    const T* col = A + (int64_t)c * lda;
    double part = 0.0;
    const int rstart = max(r0, c + 1);
    for (int r = max(r0, c - 1) + tid; r < r1; r += BS)
      if (r >= rstart) {
        const double v = col[r];
        part += v * v;
      }
    part = block_sum(part, sh);
    if (tid == 0) ws.normp[(int64_t)f * ws.MS + s] = part;
  }
}

// Step b(i): reflector of column j0+i (every segment computes the same
// scalars), scale the segment's part of it, publish dot partials.
template <typename T>
__global__ __launch_bounds__(BS) void k_qrp_b(const QRDesc* __restrict__ D, int j0, int i, QRWork ws) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  if (i >= kb) return;
  const int f = blockIdx.x, s = blockIdx.y;
  const int m = d.m;
  const int r0 = max(j0, s * RS), r1 = min(m, (s + 1) * RS);
  if (r0 >= r1) return;
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int c = j0 + i;
  double xn2 = 0.0;
  for (int sg = seg_lo(j0); sg < seg_hi(m); ++sg) xn2 += ws.normp[(int64_t)f * ws.MS + sg];
  T* col = A + (int64_t)c * lda;
  const double alpha = col[c];
  double beta, tv, scal;
  house_scalars(alpha, xn2, beta, tv, scal);
  const int rs = max(r0, c + 1);
  if (tv != 0.0)
    for (int r = rs + tid; r < r1; r += BS) col[r] = static_cast<T>(col[r] * scal);
  __syncthreads();
  const bool has_c = c >= r0 && c < r1;
  for (int cc = c + 1 + wv; cc < j0 + kb; cc += 4) {
    const T* y = A + (int64_t)cc * lda;
    double dot = 0.0;
    for (int r = rs + lane; r < r1; r += 64) dot += (double)col[r] * (double)y[r];
    dot = wave_sum(dot);
    if (lane == 0) ws.dp[((int64_t)f * ws.MS + s) * NB + (cc - j0)] = dot + (has_c ? (double)y[c] : 0.0);
  }
  if (has_c && tid == 0) {
    static_cast<T*>(d.tau)[c] = static_cast<T>(tv);
    ws.betas[f] = beta;
  }
}

// Gram partials of the panel's reflectors over the segment.
template <typename T>
__global__ __launch_bounds__(BS) void k_qrp_gram(const QRDesc* __restrict__ D, int j0, QRWork ws) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  const int f = blockIdx.x, s = blockIdx.y;
  const int m = d.m;
  const int r0 = max(j0, s * RS), r1 = min(m, (s + 1) * RS);
  if (r0 >= r1) return;
  const T* A = static_cast<const T*>(d.A);
  const int64_t lda = d.lda;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  double* gp = ws.gp + ((int64_t)f * ws.MS + s) * NB * NB;
  __shared__ double Vs[64][NB + 1];
  double acc4[4];
  gram_rows(A, lda, j0, kb, r0, r1, Vs, acc4);
  const int a = tid >> 3, b0 = (tid & 7) * 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) gp[a * NB + b0 + k] = acc4[k];
  (void)wv;
  (void)lane;
}

template <typename T>
__global__ __launch_bounds__(BS) void k_qrp_tmat(const QRDesc* __restrict__ D, int j0, QRWork ws) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  const int f = blockIdx.x;
  __shared__ double G[NB][NB + 1];
  __shared__ double s_tau[NB];
  __shared__ double Ts[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += BS) {
    const int a = e / NB, b = e % NB;
    double acc = 0.0;
    if (a < b && b < kb)
      for (int sg = seg_lo(j0); sg < seg_hi(d.m); ++sg) acc += ws.gp[((int64_t)f * ws.MS + sg) * NB * NB + e];
    G[a][b] = acc;
  }
  if (threadIdx.x < kb) s_tau[threadIdx.x] = (double)static_cast<const T*>(d.tau)[j0 + threadIdx.x];
  __syncthreads();
  build_t(ws.tbuf + (int64_t)f * NB * NB, s_tau, G, kb, Ts);
}

// ---------------------------------------------------------------------------
// trailing update
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T vref(const T* A, int64_t lda, int j0, int a, int kb, int r) {
  if (a >= kb) return T(0);
  const int ra = j0 + a;
  if (r == ra) return T(1);
  if (r > ra) return A[r + (int64_t)ra * lda];
  return T(0);
}

// W_s = V_s^T C_s for one (front, tile, segment)
template <typename T>
__global__ __launch_bounds__(BS) void k_qru_w(const QRDesc* __restrict__ D, int j0, QRWork ws) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  const int t = blockIdx.y, s = blockIdx.z;
  const int c0 = j0 + kb + t * TN;
  if (c0 >= d.n) return;
  const int m = d.m;
  const int r0 = max(j0, s * RS), r1 = min(m, (s + 1) * RS);
  if (r0 >= r1) return;
  const int nc = min(TN, d.n - c0);
  const T* A = static_cast<const T*>(d.A);
  const int64_t lda = d.lda;
  const int tid = threadIdx.x;
  __shared__ T Vs[32][NB + 1];
  __shared__ T Cs[32][TN + 1];
  const int pa = tid >> 3, pcg = tid & 7;
  double acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;
  for (int rb = r0; rb < r1; rb += 32) {
    for (int e = tid; e < 32 * NB; e += BS) {
      const int rr = e & 31, a = e >> 5;
      const int r = rb + rr;
      Vs[rr][a] = r < r1 ? vref(A, lda, j0, a, kb, r) : T(0);
    }
    for (int e = tid; e < 32 * TN; e += BS) {
      const int rr = e & 31, cc = e >> 5;
      const int r = rb + rr;
      Cs[rr][cc] = (r < r1 && cc < nc) ? A[r + (int64_t)(c0 + cc) * lda] : T(0);
    }
    __syncthreads();
    if (pa < kb) {
      const int rmax = min(32, r1 - rb);
      for (int rr = 0; rr < rmax; ++rr) {
        const double v = Vs[rr][pa];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += v * (double)Cs[rr][pcg * 8 + j];
      }
    }
    __syncthreads();
  }
  double* out = ws.wp + (((int64_t)blockIdx.x * ws.MT + t) * ws.MS + s) * NB * TN;
#pragma unroll
  for (int j = 0; j < 8; ++j) out[pa * TN + pcg * 8 + j] = acc[j];
}

// W = T^T sum_s W_s for one (front, tile)
template <typename T>
__global__ __launch_bounds__(BS) void k_qru_reduce(const QRDesc* __restrict__ D, int j0, QRWork ws) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  const int t = blockIdx.y;
  const int c0 = j0 + kb + t * TN;
  if (c0 >= d.n) return;
  __shared__ double W[NB][TN + 1];
  const int tid = threadIdx.x;
  const int64_t base = ((int64_t)blockIdx.x * ws.MT + t) * ws.MS;
  for (int e = tid; e < NB * TN; e += BS) {
    double acc = 0.0;
    for (int sg = seg_lo(j0); sg < seg_hi(d.m); ++sg) acc += ws.wp[(base + sg) * NB * TN + e];
    W[e / TN][e % TN] = acc;
  }
  __syncthreads();
  const double* Tm = ws.tbuf + (int64_t)blockIdx.x * NB * NB;
  double* out = ws.w + ((int64_t)blockIdx.x * ws.MT + t) * NB * TN;
  for (int e = tid; e < NB * TN; e += BS) {
    const int i = e / TN, cc = e % TN;
    double s = 0.0;
    if (i < kb)
      for (int a = 0; a <= i; ++a) s += Tm[a * NB + i] * W[a][cc];
    out[e] = s;
  }
}

// C_s -= V_s W for one (front, tile, segment)
template <typename T>
__global__ __launch_bounds__(BS) void k_qru_apply(const QRDesc* __restrict__ D, int j0, QRWork ws) {
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  const int t = blockIdx.y, s = blockIdx.z;
  const int c0 = j0 + kb + t * TN;
  if (c0 >= d.n) return;
  const int m = d.m;
  const int r0 = max(j0, s * RS), r1 = min(m, (s + 1) * RS);
  if (r0 >= r1) return;
  const int nc = min(TN, d.n - c0);
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int tid = threadIdx.x;
  __shared__ double W[NB][TN + 1];
  __shared__ T Vs[32][NB + 1];
  const double* win = ws.w + ((int64_t)blockIdx.x * ws.MT + t) * NB * TN;
  for (int e = tid; e < NB * TN; e += BS) W[e / TN][e % TN] = win[e];
  const int rr = tid & 31, cg = tid >> 5;
  for (int rb = r0; rb < r1; rb += 32) {
    __syncthreads();
    for (int e = tid; e < 32 * NB; e += BS) {
      const int r2 = e & 31, a = e >> 5;
      const int r = rb + r2;
      Vs[r2][a] = r < r1 ? vref(A, lda, j0, a, kb, r) : T(0);
    }
    __syncthreads();
    const int r = rb + rr;
    if (r < r1) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int cc = cg * 8 + j;
        if (cc < nc) {
          double sum = 0.0;
          for (int a = 0; a < kb; ++a) sum += (double)Vs[rr][a] * W[a][cc];
          T* p = A + r + (int64_t)(c0 + cc) * lda;
          *p = static_cast<T>((double)*p - sum);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// trailing update on the matrix cores
//
// v_mfma_f32_16x16x4f32 (FP32 fronts) and v_mfma_f64_16x16x4f64 (FP64
// fronts), one 16x16 block per wave: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] (K = 4), and holds D[row(l / 16, v)][l % 16] in
// accumulator v, with row(g, v) = 4 g + v for FP32 and g + 4 v for FP64
// (measured).  Accumulation in the storage type.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f32x4 acc;
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int g, int v) { return g + 4 * v; }
};

// W_s = V_s^T C_s for one (front, 64-column tile, row segment): output
// 32 x 64; wave w computes a-rows 16 (w & 1) .. +16 and two 16-column
// blocks 2 (w >> 1), 2 (w >> 1) + 1, over 64-row slabs staged in LDS.
template <typename T>
__global__ __launch_bounds__(BS) void k_qru_w_mfma(const QRDesc* __restrict__ D, int j0, QRWork ws) {
  typedef typename Mfma<T>::acc accT;
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  const int t = blockIdx.y, s = blockIdx.z;
  const int c0 = j0 + kb + t * TN;
  if (c0 >= d.n) return;
  const int m = d.m;
  const int r0 = max(j0, s * RS), r1 = min(m, (s + 1) * RS);
  if (r0 >= r1) return;
  const int nc = min(TN, d.n - c0);
  const T* A = static_cast<const T*>(d.A);
  const int64_t lda = d.lda;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  __shared__ T Vs[64][NB + 1];
  __shared__ T Cs[64][TN + 1];
  const int ab = wv & 1, jb = 2 * (wv >> 1);
  const int li = lane & 15, lk = lane >> 4;
  accT acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  // the next 64-row slab is fetched into registers while the current one
  // is multiplied out of LDS
  T vr[64 * NB / BS], cr[64 * TN / BS];
  auto fetch = [&](int rb) {
#pragma unroll
    for (int u = 0; u < 64 * NB / BS; ++u) {
      const int e = tid + u * BS, rr = e & 63, a = e >> 6, r = rb + rr;
      vr[u] = r < r1 ? vref(A, lda, j0, a, kb, r) : T(0);
    }
#pragma unroll
    for (int u = 0; u < 64 * TN / BS; ++u) {
      const int e = tid + u * BS, rr = e & 63, cc = e >> 6, r = rb + rr;
      cr[u] = (r < r1 && cc < nc) ? A[r + (int64_t)(c0 + cc) * lda] : T(0);
    }
  };
  fetch(r0);
  for (int rb = r0; rb < r1; rb += 64) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 64 * NB / BS; ++u) {
      const int e = tid + u * BS;
      Vs[e & 63][e >> 6] = vr[u];
    }
#pragma unroll
    for (int u = 0; u < 64 * TN / BS; ++u) {
      const int e = tid + u * BS;
      Cs[e & 63][e >> 6] = cr[u];
    }
    __syncthreads();
    if (rb + 64 < r1) fetch(rb + 64);
#pragma unroll
    for (int k4 = 0; k4 < 16; ++k4) {
      const int rr = 4 * k4 + lk;
      const T av = Vs[rr][16 * ab + li];
      acc0 = Mfma<T>::mma(av, Cs[rr][16 * jb + li], acc0);
      acc1 = Mfma<T>::mma(av, Cs[rr][16 * (jb + 1) + li], acc1);
    }
  }
  double* out = ws.wp + (((int64_t)blockIdx.x * ws.MT + t) * ws.MS + s) * NB * TN;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = 16 * ab + Mfma<T>::row(lk, v);
    out[a * TN + 16 * jb + li] = (double)acc0[v];
    out[a * TN + 16 * (jb + 1) + li] = (double)acc1[v];
  }
}

// C_s -= V_s W for one (front, 64-column tile, row segment), computed as
// (W^T V_s^T)^T so that a lane's accumulators run along rows: wave w owns
// columns 16 w .. +16 of the tile and the four 16-row blocks of each
// 64-row slab; K = kb <= 32 in steps of 4.
template <typename T>
__global__ __launch_bounds__(BS) void k_qru_apply_mfma(const QRDesc* __restrict__ D, int j0, QRWork ws) {
  typedef typename Mfma<T>::acc accT;
  const QRDesc d = D[blockIdx.x];
  const int kk = min(d.m, d.k);
  if (j0 >= kk) return;
  const int kb = min(NB, kk - j0);
  const int t = blockIdx.y, s = blockIdx.z;
  const int c0 = j0 + kb + t * TN;
  if (c0 >= d.n) return;
  const int m = d.m;
  const int r0 = max(j0, s * RS), r1 = min(m, (s + 1) * RS);
  if (r0 >= r1) return;
  const int nc = min(TN, d.n - c0);
  T* A = static_cast<T*>(d.A);
  const int64_t lda = d.lda;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  __shared__ T Ws[NB][TN + 1];
  __shared__ T Vs[64][NB + 1];
  const double* win = ws.w + ((int64_t)blockIdx.x * ws.MT + t) * NB * TN;
  for (int e = tid; e < NB * TN; e += BS) Ws[e / TN][e % TN] = static_cast<T>(win[e]);
  const int li = lane & 15, lk = lane >> 4;
  int col[4];  // this lane's four columns of the tile
#pragma unroll
  for (int v = 0; v < 4; ++v) col[v] = 16 * wv + Mfma<T>::row(lk, v);
  // The next slab's reflector rows and this lane's 16 entries of C are
  // fetched into registers while the current slab is multiplied.
  T vr[64 * NB / BS], cr[4][4];
  auto fetch = [&](int rb) {
#pragma unroll
    for (int u = 0; u < 64 * NB / BS; ++u) {
      const int e = tid + u * BS, rr = e & 63, a = e >> 6, r = rb + rr;
      vr[u] = r < r1 ? vref(A, lda, j0, a, kb, r) : T(0);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = rb + 16 * b + li;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cr[b][v] = (r < r1 && col[v] < nc) ? A[r + (int64_t)(c0 + col[v]) * lda] : T(0);
    }
  };
  fetch(r0);
  for (int rb = r0; rb < r1; rb += 64) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 64 * NB / BS; ++u) {
      const int e = tid + u * BS;
      Vs[e & 63][e >> 6] = vr[u];
    }
    T cc[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) cc[b][v] = cr[b][v];
    __syncthreads();
    if (rb + 64 < r1) fetch(rb + 64);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      accT acc = {0, 0, 0, 0};
#pragma unroll
      for (int k4 = 0; k4 < NB / 4; ++k4) {
        const int a = 4 * k4 + lk;
        acc = Mfma<T>::mma(Ws[a][16 * wv + li], Vs[16 * b + li][a], acc);
      }
      const int r = rb + 16 * b + li;
      if (r < r1)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (col[v] < nc) A[r + (int64_t)(c0 + col[v]) * lda] = cc[b][v] - acc[v];
    }
  }
}

}  // namespace

void qr_work_dims(const std::vector<QRDesc>& h, int* MS, int* MT) {
  int ms = 1, mt = 1;
  for (auto& d : h) {
    ms = std::max(ms, (d.m + RS - 1) / RS);
    const int kk = std::min(d.m, d.k);
    if (kk > 0) mt = std::max(mt, (d.n - std::min(NB, kk) + TN - 1) / TN);
  }
  *MS = ms;
  *MT = std::max(1, mt);
}

template <typename T>
void launch_qr(const QRDesc* d_desc, const std::vector<QRDesc>& h, const QRWork& ws, hipStream_t s,
               int* launches, KernelTimer* kt, bool allow_coop) {
  if (h.empty()) return;
  const unsigned nf = (unsigned)h.size();
  int kmax = 0, mmax = 0;
  for (auto& d : h) {
    kmax = std::max(kmax, std::min(d.m, d.k));
    mmax = std::max(mmax, d.m);
  }
  // tall fronts: row-split panels
  const bool split = mmax > 2 * RS;
  for (int j0 = 0; j0 < kmax; j0 += NB) {
    int tiles = 0, segs = 1, kbmax = 0;
    for (auto& d : h) {
      const int kk = std::min(d.m, d.k);
      if (j0 >= kk) continue;
      const int kb = std::min(NB, kk - j0);
      kbmax = std::max(kbmax, kb);
      const int rest = d.n - j0 - kb;
      if (rest > 0) tiles = std::max(tiles, (rest + TN - 1) / TN);
      segs = std::max(segs, (d.m + RS - 1) / RS);
    }
    int coop_segs = 0;
    // SPAQR_NO_COOP=1 keeps tall panels on the two-launches-per-column path
    // (for tools that cannot follow cooperative launches)
    static const bool no_coop = std::getenv("SPAQR_NO_COOP") != nullptr;
    if (split && !no_coop && allow_coop) {
      constexpr int TSEG = CoopRows<T>::TSEG;
      coop_segs = (mmax - j0 + TSEG - 1) / TSEG;
      static int max_coop = -1;  // per storage type
      if (max_coop < 0) {
        int per_cu = 0, dev = 0, cus = 0;
        SPAQR_HIP(hipGetDevice(&dev));
        SPAQR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        SPAQR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_qrp_coop<T>, PBS, 0));
        max_coop = per_cu * cus;
      }
      if ((int64_t)nf * coop_segs > max_coop || coop_segs > ws.MS) coop_segs = 0;
    }
    if (coop_segs > 0) {
      const QRDesc* dd = d_desc;
      int a_j0 = j0, a_kb = kbmax, a_s = coop_segs;
      QRWork a_ws = ws;
      void* args[] = {(void*)&dd, (void*)&a_j0, (void*)&a_kb, (void*)&a_s, (void*)&a_ws};
      const bool timed = kt && kt->pick("qrp_coop");
      if (timed) kt->mark(s);
      SPAQR_HIP(hipLaunchCooperativeKernel((const void*)k_qrp_coop<T>, dim3(nf * coop_segs), dim3(PBS), args, 0, s));
      if (timed) {
        kt->close(s);
        // algorithmic work of the panel: Householder QR of (m - j0) x kb,
        // the panel read and written once
        for (auto& d : h) {
          const int kk = std::min(d.m, d.k);
          if (j0 >= kk) continue;
          const double mr = d.m - j0, kb = std::min(NB, kk - j0);
          kt->flops += 2.0 * mr * kb * kb - 2.0 * kb * kb * kb / 3.0;
          kt->bytes += 2.0 * sizeof(T) * mr * kb;
        }
      }
      ++*launches;
    } else if (split) {
      const dim3 g(nf, segs);
      for (int i = 0; i <= kbmax; ++i) {
        hipLaunchKernelGGL(k_qrp_a<T>, g, dim3(BS), 0, s, d_desc, j0, i, ws);
        ++*launches;
        if (i < kbmax) {
          hipLaunchKernelGGL(k_qrp_b<T>, g, dim3(BS), 0, s, d_desc, j0, i, ws);
          ++*launches;
        }
      }
      hipLaunchKernelGGL(k_qrp_gram<T>, g, dim3(BS), 0, s, d_desc, j0, ws);
      hipLaunchKernelGGL(k_qrp_tmat<T>, dim3(nf), dim3(BS), 0, s, d_desc, j0, ws);
      *launches += 2;
    } else if (sizeof(T) == 4 && mmax - j0 <= PBS * PRPT) {
      hipLaunchKernelGGL(k_qr_panel_reg, dim3(nf), dim3(PBS), 0, s, d_desc, j0, ws.tbuf);
      ++*launches;
    } else {
      hipLaunchKernelGGL(k_qr_panel<T>, dim3(nf), dim3(BS), 0, s, d_desc, j0, ws.tbuf);
      ++*launches;
    }
    SPAQR_HIP(hipGetLastError());
    if (tiles > 0) {
      const dim3 g3(nf, tiles, segs), g2(nf, tiles);
      // SPAQR_VALU_UPDATE=1 keeps FP64 fronts on the vector-ALU update
      // (for comparisons with the matrix-core form)
      static const bool valu64 = std::getenv("SPAQR_VALU_UPDATE") != nullptr;
      const bool mfma = sizeof(T) == 4 || !valu64;
      if (mfma)
        hipLaunchKernelGGL(k_qru_w_mfma<T>, g3, dim3(BS), 0, s, d_desc, j0, ws);
      else
        hipLaunchKernelGGL(k_qru_w<T>, g3, dim3(BS), 0, s, d_desc, j0, ws);
      hipLaunchKernelGGL(k_qru_reduce<T>, g2, dim3(BS), 0, s, d_desc, j0, ws);
      if (mfma)
        hipLaunchKernelGGL(k_qru_apply_mfma<T>, g3, dim3(BS), 0, s, d_desc, j0, ws);
      else
        hipLaunchKernelGGL(k_qru_apply<T>, g3, dim3(BS), 0, s, d_desc, j0, ws);
      SPAQR_HIP(hipGetLastError());
      *launches += 3;
    }
  }
}

template void launch_qr<double>(const QRDesc*, const std::vector<QRDesc>&, const QRWork&, hipStream_t, int*,
                                KernelTimer*, bool);
template void launch_qr<float>(const QRDesc*, const std::vector<QRDesc>&, const QRWork&, hipStream_t, int*,
                               KernelTimer*, bool);

}  // namespace spaqr
