// The handle behind spaqr_handle: the host plan, device copies of the
// matrix, the factor (device ops + host metadata) and solver workspace.
#pragma once

#include <string>
#include <vector>

#include "spaqr_impl.h"

struct spaqr_handle_s;

namespace spaqr {

struct OpRec {
  int kind = 0;   // 0 eliminate, 1 scale, 2 sparsify
  int level = 0, round = 0, phase = 0;
  const void* R = nullptr;
  const void* tau = nullptr;
  int64_t ld = 0;
  int n1 = 0, n2 = 0;
  const int* d_s1 = nullptr;
  const int* d_s2 = nullptr;
  std::vector<int> s1, s2;
};

struct ApplyBatch {
  const ApplyOp* d_ops = nullptr;
  int n = 0;
  int max_n1 = 0;
};

struct Handle {
  std::string err;
  spaqr_options opt{};
  Plan P;
  hipStream_t stream = nullptr;
  bool dev_ready = false;
  // device copies of the matrix (scaled values A D^-1 and its transpose)
  double* d_ahat = nullptr;
  int64_t* d_rp = nullptr;
  int32_t* d_ci = nullptr;
  double* d_ahatT = nullptr;
  int64_t* d_atp = nullptr;
  int32_t* d_ati = nullptr;
  int64_t* d_init_dst = nullptr;
  double* d_D = nullptr;
  size_t plan_bytes = 0;
  // factor
  Arena arena;
  Staging stage;
  bool factored = false;
  int precision = SPAQR_FP64;
  std::vector<OpRec> ops;
  std::vector<ApplyBatch> batches;
  std::vector<int> ranks;
  spaqr_stats stats{};
  // solver workspace
  double* d_cg = nullptr;
  size_t cg_elems = 0;
  double* h_sc = nullptr;  // pinned scalars

  ~Handle();
  void ensure_device();
  void release_device();
};

void factorize(Handle& H, double eps, const int* forced, int nforced);
void apply_op(Handle& H, bool transpose, double* x_dev);
int cgls(Handle& H, const double* b, double tol, int max_iter, double* x, spaqr_cgls_info* info);
void csne(Handle& H, const double* b, double* x);

}  // namespace spaqr
