// extern "C" boundary of libspaqr: argument checks, error capture, and
// dispatch into the host analysis, the device factorization and the
// solvers.  No C++ exception leaves this file.
#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "handle.h"

struct spaqr_handle_s {
  spaqr::Handle h;
};

namespace {

thread_local std::string g_err;

template <class F>
int guard(spaqr_handle h, F&& f) {
  try {
    return f();
  } catch (const spaqr::Error& e) {
    (h ? h->h.err : g_err) = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    (h ? h->h.err : g_err) = "host allocation failed";
    return SPAQR_ENOMEM;
  } catch (const std::exception& e) {
    (h ? h->h.err : g_err) = e.what();
    return SPAQR_EARG;
  } catch (...) {
    (h ? h->h.err : g_err) = "unknown error";
    return SPAQR_EARG;
  }
}

}  // namespace

extern "C" {

int spaqr_analyze(const int64_t* row_ptr, const int32_t* col_idx, const double* vals, int64_t M,
                  int64_t N, const spaqr_options* opt, spaqr_handle* out) {
  return guard(nullptr, [&]() -> int {
    if (!out || !opt) throw spaqr::Error(SPAQR_EARG, "null argument");
    *out = nullptr;
    if (opt->precision != SPAQR_FP64 && opt->precision != SPAQR_FP32_FACTOR)
      throw spaqr::Error(SPAQR_EARG, "unknown precision");
    std::unique_ptr<spaqr_handle_s> h(new spaqr_handle_s());
    h->h.opt = *opt;
    spaqr::analyze_plan(h->h.P, row_ptr, col_idx, vals, M, N, *opt);
    *out = h.release();
    return SPAQR_OK;
  });
}

int spaqr_get_ordering(spaqr_handle h, int32_t* col_perm, int32_t* row_owner) {
  return guard(h, [&]() -> int {
    if (!h) throw spaqr::Error(SPAQR_EARG, "null handle");
    const spaqr::Plan& P = h->h.P;
    if (col_perm) {
      int64_t k = 0;
      for (int f : P.finest)
        for (int j : P.clusters[f].cells) col_perm[k++] = j;
    }
    if (row_owner)
      for (int64_t r = 0; r < P.M; ++r) row_owner[r] = P.clusters[P.row_owner[r]].finest_index;
    return SPAQR_OK;
  });
}

int spaqr_set_values(spaqr_handle h, const double* vals_dev) {
  return guard(h, [&]() -> int {
    if (!h || !vals_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    spaqr::Handle& H = h->h;
    H.ensure_device();
    H.factored = false;
    SPAQR_HIP(hipMemcpyAsync(H.d_vals, vals_dev, H.P.nnz * sizeof(double), hipMemcpyDeviceToDevice,
                             H.stream));
    spaqr::scale_values(H);
    return SPAQR_OK;
  });
}

int spaqr_factorize(spaqr_handle h, double eps) {
  return guard(h, [&]() -> int {
    if (!h) throw spaqr::Error(SPAQR_EARG, "null handle");
    spaqr::factorize(h->h, eps, nullptr, 0);
    return SPAQR_OK;
  });
}

int spaqr_factorize_forced(spaqr_handle h, double eps, const int32_t* ranks, int32_t nranks) {
  return guard(h, [&]() -> int {
    if (!h || (!ranks && nranks > 0) || nranks < 0) throw spaqr::Error(SPAQR_EARG, "bad argument");
    static const int32_t none = 0;
    spaqr::factorize(h->h, eps, ranks ? ranks : &none, nranks);
    return SPAQR_OK;
  });
}

int spaqr_apply(spaqr_handle h, const double* b_dev, double* x_dev) {
  return guard(h, [&]() -> int {
    if (!h || !b_dev || !x_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    spaqr::csne(h->h, b_dev, x_dev);
    return SPAQR_OK;
  });
}

int spaqr_csne(spaqr_handle h, const double* b_dev, double tol, int32_t max_steps, double* x_dev,
               spaqr_cgls_info* info) {
  return guard(h, [&]() -> int {
    if (!h || !b_dev || !x_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    std::vector<spaqr_cgls_info> all(h->h.P.count);
    const int rc = spaqr::csne_refine(h->h, b_dev, tol, max_steps, x_dev, all.data());
    if (info) {
      // a batch reports its worst problem
      spaqr_cgls_info w = all[0];
      for (const auto& i : all)
        if (i.residual > w.residual) w = i;
      *info = w;
    }
    return rc;
  });
}

int spaqr_autotune(spaqr_handle h, double eps, int32_t reps, const char* cache_path, spaqr_tune* out) {
  return guard(h, [&]() -> int {
    if (!h) throw spaqr::Error(SPAQR_EARG, "null handle");
    spaqr::autotune(h->h, eps, reps, cache_path, out);
    return SPAQR_OK;
  });
}

int spaqr_set_tune(spaqr_handle h, const spaqr_tune* t) {
  return guard(h, [&]() -> int {
    if (!h || !t) throw spaqr::Error(SPAQR_EARG, "null argument");
    spaqr::TuneParams p;
    p.pqr_poll = t->pqr_poll;
    p.pqr_reg_rows = t->pqr_reg_rows;
    p.tall_coop = t->tall_coop;
    spaqr::check_tune(p);
    h->h.tune = p;
    return SPAQR_OK;
  });
}

int spaqr_get_tune(spaqr_handle h, spaqr_tune* out) {
  return guard(h, [&]() -> int {
    if (!h || !out) throw spaqr::Error(SPAQR_EARG, "null argument");
    *out = spaqr_tune{};
    out->pqr_poll = h->h.tune.pqr_poll;
    out->pqr_reg_rows = h->h.tune.pqr_reg_rows;
    out->tall_coop = h->h.tune.tall_coop;
    return SPAQR_OK;
  });
}

int spaqr_apply_noalloc(spaqr_handle h, const double* b_dev, double* x_dev) {
  return guard(h, [&]() -> int {
    if (!h || !b_dev || !x_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    spaqr::csne_noalloc(h->h, b_dev, x_dev);
    return SPAQR_OK;
  });
}

int spaqr_apply_op(spaqr_handle h, int32_t op, const double* in_dev, double* out_dev) {
  return guard(h, [&]() -> int {
    if (!h || !in_dev || !out_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    if (op != SPAQR_WINV && op != SPAQR_WINVT) throw spaqr::Error(SPAQR_EARG, "unknown op");
    spaqr::Handle& H = h->h;
    if (!H.factored) throw spaqr::Error(SPAQR_ESTATE, "factorize first");
    if (in_dev != out_dev)
      SPAQR_HIP(hipMemcpyAsync(out_dev, in_dev, H.P.N * sizeof(double), hipMemcpyDeviceToDevice, H.stream));
    spaqr::apply_op(H, op == SPAQR_WINVT, out_dev);
    SPAQR_HIP(hipStreamSynchronize(H.stream));
    H.kt.harvest();
    return SPAQR_OK;
  });
}

int spaqr_cgls(spaqr_handle h, const double* b_dev, double tol, int32_t max_iter, double* x_dev,
               spaqr_cgls_info* info) {
  return guard(h, [&]() -> int {
    if (!h || !b_dev || !x_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    std::vector<spaqr_cgls_info> all(h->h.P.count);
    const int rc = spaqr::cgls(h->h, b_dev, tol, max_iter, x_dev, all.data());
    if (info) {
      // a batch reports its worst member
      spaqr_cgls_info w = all[0];
      for (const auto& a : all) {
        w.iters = std::max(w.iters, a.iters);
        w.converged = w.converged && a.converged;
        w.residual = std::max(w.residual, a.residual);
        w.paper_residual = std::max(w.paper_residual, a.paper_residual);
        w.norm_a = std::max(w.norm_a, a.norm_a);
      }
      *info = w;
    }
    return rc;
  });
}

int spaqr_batch_analyze(int32_t count, const int64_t* const* row_ptr, const int32_t* const* col_idx,
                        const double* const* vals, const int64_t* M, const int64_t* N, const spaqr_options* opts,
                        spaqr_handle* out) {
  return guard(nullptr, [&]() -> int {
    if (!out || !opts || !row_ptr || !col_idx || !vals || !M || !N || count < 1)
      throw spaqr::Error(SPAQR_EARG, "bad argument");
    *out = nullptr;
    for (int32_t g = 0; g < count; ++g) {
      const spaqr_options& o = opts[g];
      if (o.precision != opts[0].precision || o.device != opts[0].device || o.stream != opts[0].stream)
        throw spaqr::Error(SPAQR_EARG, "batch members must share precision, device and stream");
      if (o.precision != SPAQR_FP64 && o.precision != SPAQR_FP32_FACTOR)
        throw spaqr::Error(SPAQR_EARG, "unknown precision");
    }
    std::vector<spaqr::Plan> parts(count);
    for (int32_t g = 0; g < count; ++g) {
      try {
        spaqr::analyze_plan(parts[g], row_ptr[g], col_idx[g], vals[g], M[g], N[g], opts[g]);
      } catch (const spaqr::Error& e) {
        throw spaqr::Error(e.code, "batch member " + std::to_string(g) + ": " + e.what());
      }
    }
    std::unique_ptr<spaqr_handle_s> h(new spaqr_handle_s());
    h->h.opt = opts[0];
    spaqr::union_plans(h->h.P, parts);
    *out = h.release();
    return SPAQR_OK;
  });
}

int spaqr_batch_info(spaqr_handle h, int32_t* count, int64_t* col_off, int64_t* row_off) {
  return guard(h, [&]() -> int {
    if (!h || !count) throw spaqr::Error(SPAQR_EARG, "null argument");
    const spaqr::Plan& P = h->h.P;
    *count = P.count;
    for (int g = 0; g <= P.count; ++g) {
      if (col_off) col_off[g] = P.seg_col[g];
      if (row_off) row_off[g] = P.seg_row[g];
    }
    return SPAQR_OK;
  });
}

int spaqr_batch_cgls(spaqr_handle h, const double* b_dev, double tol, int32_t max_iter, double* x_dev,
                     spaqr_cgls_info* infos) {
  return guard(h, [&]() -> int {
    if (!h || !b_dev || !x_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    return spaqr::cgls(h->h, b_dev, tol, max_iter, x_dev, infos);
  });
}

int spaqr_adjoint(spaqr_handle h, const double* x_dev, const double* b_dev, const double* g_dev,
                  double tol, int32_t max_iter, double* grad_b_dev, double* grad_vals_dev,
                  double* lambda_dev, spaqr_cgls_info* info) {
  return guard(h, [&]() -> int {
    if (!h || !g_dev) throw spaqr::Error(SPAQR_EARG, "null argument");
    if (grad_vals_dev && (!x_dev || !b_dev)) throw spaqr::Error(SPAQR_EARG, "grad_vals needs x and b");
    return spaqr::adjoint(h->h, x_dev, b_dev, g_dev, tol, max_iter, grad_b_dev, grad_vals_dev, lambda_dev,
                          info);
  });
}

int spaqr_factor_stats(spaqr_handle h, spaqr_stats* out) {
  return guard(h, [&]() -> int {
    if (!h || !out) throw spaqr::Error(SPAQR_EARG, "null argument");
    if (!h->h.factored) throw spaqr::Error(SPAQR_ESTATE, "factorize first");
    *out = h->h.stats;
    out->kernel_calls = h->h.kt.calls;
    out->kernel_seconds = h->h.kt.seconds;
    out->kernel_bytes = h->h.kt.bytes;
    out->kernel_flops = h->h.kt.flops;
    out->kernel_span_calls = h->h.kt.span_calls;
    out->kernel_span_seconds = h->h.kt.span_seconds;
    return SPAQR_OK;
  });
}

int spaqr_time_kernel(spaqr_handle h, const char* family, int32_t every) {
  return guard(h, [&]() -> int {
    if (!h) throw spaqr::Error(SPAQR_EARG, "null handle");
    const std::string f = family ? family : "";
    if (!f.empty() && f != "pqr_step" && f != "apply" && f != "qrp_coop")
      throw spaqr::Error(SPAQR_EARG, "unknown kernel family '" + f + "'");
    if (every < 1) throw spaqr::Error(SPAQR_EARG, "every must be >= 1");
    h->h.kt.reset(f.c_str(), every);
    return SPAQR_OK;
  });
}

int spaqr_get_ranks(spaqr_handle h, int32_t* ranks, int32_t cap, int32_t* n) {
  return guard(h, [&]() -> int {
    if (!h || !n) throw spaqr::Error(SPAQR_EARG, "null argument");
    if (!h->h.factored) throw spaqr::Error(SPAQR_ESTATE, "factorize first");
    const auto& r = h->h.ranks;
    *n = (int32_t)r.size();
    if (ranks)
      for (int32_t i = 0; i < cap && i < (int32_t)r.size(); ++i) ranks[i] = r[i];
    return SPAQR_OK;
  });
}

int spaqr_get_op(spaqr_handle h, int32_t i, spaqr_op_desc* desc, double* mat, int32_t* slots1,
                 int32_t* slots2, double* tau) {
  return guard(h, [&]() -> int {
    if (!h) throw spaqr::Error(SPAQR_EARG, "null handle");
    spaqr::Handle& H = h->h;
    if (!H.factored) throw spaqr::Error(SPAQR_ESTATE, "factorize first");
    if (i < 0 || i >= (int32_t)H.ops.size()) throw spaqr::Error(SPAQR_EARG, "op index out of range");
    const spaqr::OpRec& o = H.ops[i];
    if (desc) {
      desc->kind = o.kind;
      desc->n1 = o.n1;
      desc->n2 = o.kind == 1 ? 0 : o.n2;
      desc->round = o.round;
      desc->level = o.level;
    }
    if (slots1)
      for (size_t k = 0; k < o.s1.size(); ++k) slots1[k] = o.s1[k];
    if (slots2)
      for (size_t k = 0; k < o.s2.size(); ++k) slots2[k] = o.s2[k];
    const size_t es = H.precision == SPAQR_FP32_FACTOR ? 4 : 8;
    auto fetch = [&](const void* src, int64_t ld, int rows, int cols, std::vector<double>& out) {
      std::vector<char> raw((size_t)ld * cols * es);
      if (!raw.empty())
        SPAQR_HIP(hipMemcpy(raw.data(), src, raw.size(), hipMemcpyDeviceToHost));
      out.assign((size_t)rows * cols, 0.0);
      for (int c = 0; c < cols; ++c)
        for (int r = 0; r < rows; ++r) {
          const size_t k = (size_t)r + (size_t)c * ld;
          out[(size_t)r * cols + c] =
              es == 4 ? (double)reinterpret_cast<const float*>(raw.data())[k] : reinterpret_cast<const double*>(raw.data())[k];
        }
    };
    if (mat || tau) {
      SPAQR_HIP(hipStreamSynchronize(H.stream));
      std::vector<double> m;
      if (o.kind == 0) {
        fetch(o.R, o.ld, o.n1, o.n1 + o.n2, m);
        for (int r = 0; r < o.n1; ++r)
          for (int c = 0; c < r; ++c) m[(size_t)r * (o.n1 + o.n2) + c] = 0.0;
      } else if (o.kind == 1) {
        fetch(o.R, o.ld, o.n1, o.n1, m);
        for (int r = 0; r < o.n1; ++r)
          for (int c = 0; c < r; ++c) m[(size_t)r * o.n1 + c] = 0.0;
      } else {
        fetch(o.R, o.ld, o.n1, o.n2, m);
      }
      if (mat) std::memcpy(mat, m.data(), m.size() * sizeof(double));
      if (tau && o.kind == 2 && o.n2 > 0) {
        std::vector<double> t;
        fetch(o.tau, 1, 1, o.n2, t);
        std::memcpy(tau, t.data(), t.size() * sizeof(double));
      }
    }
    return SPAQR_OK;
  });
}

int spaqr_destroy(spaqr_handle h) {
  if (!h) return SPAQR_OK;
  return guard(nullptr, [&]() -> int {
    delete h;
    return SPAQR_OK;
  });
}

const char* spaqr_last_error(spaqr_handle h) { return h ? h->h.err.c_str() : g_err.c_str(); }

}  // extern "C"
