// Autotuner of the factorization's launch shapes, per problem.
//
// Three knobs change how the same arithmetic is launched, never what is
// computed beyond rounding of the panel form:
//   * pqr_poll      pivot steps of a rank-revealing-QR batch launched ahead
//                   of the last step the GPU has reported its live-matrix
//                   count for (a deeper queue, more empty launches once every
//                   matrix has stopped);
//   * pqr_reg_rows  tallest 64-aligned row window a pivot step keeps in
//                   registers (per-lane register tile of 2 to 16 rows, or
//                   the memory path above it; both sum in the same order);
//   * tall_coop     tall Householder panels in one cooperative launch
//                   or in two launches per column.
// The tuner times whole factorizations of the handle's own problem (the
// best of `reps` runs per setting), descends one knob at a time from the
// defaults, and caches the choice in a text file keyed by the problem's
// signature, so later runs load it instead of timing again.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "handle.h"

namespace spaqr {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

std::string signature(Handle& H, double eps) {
  hipDeviceProp_t prop{};
  int dev = 0;
  SPAQR_HIP(hipGetDevice(&dev));
  SPAQR_HIP(hipGetDeviceProperties(&prop, dev));
  std::ostringstream o;
  std::string arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ') c = '_';
  o << "M=" << H.P.M << ",N=" << H.P.N << ",nnz=" << H.P.nnz << ",depth=" << H.P.depth << ",skip=" << H.P.skip
    << ",count=" << H.P.count << ",prec=" << H.opt.precision << ",eps=" << eps << ",arch=" << arch;
  return o.str();
}

double time_factorization(Handle& H, double eps, int reps) {
  double best = 1e300;
  for (int r = 0; r < reps; ++r) {
    SPAQR_HIP(hipStreamSynchronize(H.stream));
    const double t0 = now_s();
    factorize(H, eps, nullptr, 0);
    SPAQR_HIP(hipStreamSynchronize(H.stream));
    best = std::min(best, now_s() - t0);
  }
  return best;
}

}  // namespace

void check_tune(const TuneParams& t) {
  if (t.pqr_poll < 1 || t.pqr_poll > 4096) throw Error(SPAQR_EARG, "pqr_poll must be in 1..4096");
  if (t.pqr_reg_rows < 0 || t.pqr_reg_rows > 1024) throw Error(SPAQR_EARG, "pqr_reg_rows must be in 0..1024");
  if (t.tall_coop != 0 && t.tall_coop != 1) throw Error(SPAQR_EARG, "tall_coop must be 0 or 1");
}

void autotune(Handle& H, double eps, int reps, const char* cache_path, spaqr_tune* out) {
  if (reps < 1) throw Error(SPAQR_EARG, "reps must be >= 1");
  if (!(eps >= 0.0)) throw Error(SPAQR_EARG, "eps must be >= 0");
  H.ensure_device();
  const std::string sig = signature(H, eps);
  spaqr_tune res{};
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    bool found = false;
    TuneParams t;
    double sd = 0.0, sb = 0.0;
    int ev = 0;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string key;
      TuneParams c;
      double a = 0.0, b = 0.0;
      int e = 0;
      if (ls >> key >> c.pqr_poll >> c.pqr_reg_rows >> c.tall_coop >> a >> b >> e && key == sig) {
        t = c, sd = a, sb = b, ev = e;
        found = true;  // the last entry for the signature wins
      }
    }
    if (found) {
      check_tune(t);
      H.tune = t;
      res.from_cache = 1;
      res.seconds_default = sd;
      res.seconds_best = sb;
      res.evaluations = ev;
    }
  }
  if (!res.from_cache) {
    TuneParams best;  // defaults
    H.tune = best;
    const double t_def = time_factorization(H, eps, reps);
    double t_best = t_def;
    int evals = 1;
    auto consider = [&](TuneParams c) {
      H.tune = c;
      const double t = time_factorization(H, eps, reps);
      ++evals;
      if (t < t_best) t_best = t, best = c;
    };
    for (int poll : {4, 8}) {
      TuneParams c = best;
      c.pqr_poll = poll;
      consider(c);
    }
    for (int rr : {256, 512}) {
      TuneParams c = best;
      c.pqr_reg_rows = rr;
      consider(c);
    }
    {
      TuneParams c = best;
      c.tall_coop = 1 - c.tall_coop;
      consider(c);
    }
    H.tune = best;
    res.seconds_default = t_def;
    res.seconds_best = t_best;
    res.evaluations = evals;
    if (cache_path && *cache_path) {
      std::ofstream o(cache_path, std::ios::app);
      if (!o) throw Error(SPAQR_EARG, std::string("cannot write the tuning cache ") + cache_path);
      char buf[128];
      std::snprintf(buf, sizeof buf, " %d %d %d %.6e %.6e %d", best.pqr_poll, best.pqr_reg_rows, best.tall_coop,
                    t_def, t_best, evals);
      o << sig << buf << "\n";
    }
  }
  // leave the handle factored with the chosen shapes
  factorize(H, eps, nullptr, 0);
  if (out) {
    res.pqr_poll = H.tune.pqr_poll;
    res.pqr_reg_rows = H.tune.pqr_reg_rows;
    res.tall_coop = H.tune.tall_coop;
    *out = res;
  }
}

}  // namespace spaqr
