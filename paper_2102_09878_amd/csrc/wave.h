// Wave-wide (64 lanes) reductions on the DPP cross-lane paths of gfx9-class
// GPUs: no LDS round trip per level.  The summation tree is fixed (pairs,
// quads, 8- and 16-lane rows, then rows 0+1 and 2+3 and the halves), so every
// sum is reproducible; the total is read from lane 63 and returned to all
// lanes.
#pragma once

#include <hip/hip_runtime.h>

namespace spaqr {

// lanes of the DPP source pattern CTRL, in the rows of ROWMASK (0 elsewhere)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_take(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// value of lane `l` (uniform over the wave) in every lane, through SGPRs
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// the wave's total in lane 63 (the other lanes hold partial sums)
__device__ __forceinline__ double wave_sum63(double v) {
  v += dpp_take<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]: pairs
  v += dpp_take<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]: quads
  v += dpp_take<0x141, 0xf>(v);  // row_half_mirror: 8 lanes
  v += dpp_take<0x140, 0xf>(v);  // row_mirror: 16 lanes
  v += dpp_take<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_take<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  return v;
}

__device__ __forceinline__ double wave_sum_dpp(double v) { return lane63(wave_sum63(v)); }


// (v, i) with the largest v, lowest i on ties, over the wave, returned to
// all lanes.  Rows outside a step's mask see (-1, INT_MAX), which loses to
// every candidate (values are norms, >= 0, or -1 for none).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void amax_take(double& v, int& i) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)0xBFF00000, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  const int oi = __builtin_amdgcn_update_dpp(0x7fffffff, i, CTRL, ROWMASK, 0xf, false);
  const double ov = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  if (ov > v || (ov == v && oi < i)) v = ov, i = oi;
}

__device__ __forceinline__ void wave_argmax_dpp(double& v, int& i) {
  amax_take<0xB1, 0xf>(v, i);
  amax_take<0x4E, 0xf>(v, i);
  amax_take<0x141, 0xf>(v, i);
  amax_take<0x140, 0xf>(v, i);
  amax_take<0x142, 0xa>(v, i);
  amax_take<0x143, 0xc>(v, i);
  v = lane63(v);
  i = __builtin_amdgcn_readlane(i, 63);
}

}  // namespace spaqr
