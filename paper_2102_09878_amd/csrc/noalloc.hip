// One-shot seminormal solve x = D^-1 W^-1 W^-T D^-1 A^T b (the same
// operation as spaqr_apply) that allocates no device memory, for callers
// that cannot allocate: code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc.
//
// Every intermediate of the call lives in one file-scope device array,
// `scratch`, of kScratchDoubles doubles (16 MiB) that each GPU the library
// runs on holds until the process ends:
//   [ t : N slots ][ W-sweep staging : nstage ][ W-sweep chunk partials : awork ]
// each part starting on a 256-byte boundary.  The array's address is taken
// once per device, with that device current, on the first call there; host
// code only ever passes that address.  Calls on one GPU share the array,
// so calls that overlap on one GPU (two streams, two threads) race.  Every
// part is written before it is read within a call (the product A^T b
// writes all N entries of t; each sweep batch writes its staging and
// partials before reading them), so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cgls.h"
#include "handle.h"

namespace spaqr {

namespace {

constexpr int64_t kScratchDoubles = int64_t(1) << 21;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_addr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (taken once per device).
double* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(SPAQR_EARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    int cur = 0;
    SPAQR_HIP(hipGetDevice(&cur));
    if (cur != dev) SPAQR_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) SPAQR_HIP(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      throw Error(SPAQR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_addr[dev] = static_cast<double*>(p);
  }
  return g_addr[dev];
}

int64_t up256(int64_t doubles) { return (doubles + 31) / 32 * 32; }

}  // namespace

void csne_noalloc(Handle& H, const double* b, double* x) {
  if (!H.factored) throw Error(SPAQR_ESTATE, "factorize first");
  const int64_t N = H.P.N;
  const int64_t o_stage = up256(N), o_work = o_stage + up256(H.nstage_elems);
  const int64_t need = o_work + up256(H.awork_elems);
  if (need > kScratchDoubles)
    throw Error(SPAQR_EARG, "spaqr_apply_noalloc: the problem needs " + std::to_string(need) +
                                " doubles of scratch, above the limit of " + std::to_string(kScratchDoubles) +
                                " (16 MiB); use spaqr_apply");
  double* base = scratch_on(H.opt.device);
  double* t = base;
  launch_spmv(H.d_atp, H.d_ati, H.d_ahatT, b, t, N, H.stream);  // t = Ahat^T b
  apply_op(H, true, t, base + o_stage, base + o_work, false);   // W^-T
  apply_op(H, false, t, base + o_stage, base + o_work, false);  // W^-1
  launch_scale(x, t, H.d_D, N, false, H.stream);                // x = D^-1 t
  SPAQR_HIP(hipStreamSynchronize(H.stream));
}

}  // namespace spaqr
