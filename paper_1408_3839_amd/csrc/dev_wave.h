// Wave-level reductions of doubles with DPP lane moves (a few cycles each)
// instead of LDS-routed lane permutes.  Each double moves as two 32-bit
// halves with the same DPP control.  Controls (GFX9 DPP): quad_perm
// [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E, row_half_mirror = 0x141,
// row_mirror = 0x140, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
#pragma once
#include <hip/hip_runtime.h>

namespace tl {
namespace dev {

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROW_MASK,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROW_MASK,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over each group of 8 consecutive lanes; every lane of the group gets it.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_d<0xB1>(v, 0.0);
  v += dpp_d<0x4E>(v, 0.0);
  v += dpp_d<0x141>(v, 0.0);
  return v;
}

__device__ __forceinline__ double group8_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v, v));
  v = fmax(v, dpp_d<0x4E>(v, v));
  return fmax(v, dpp_d<0x141>(v, v));
}

__device__ __forceinline__ double group8_min(double v) {
  v = fmin(v, dpp_d<0xB1>(v, v));
  v = fmin(v, dpp_d<0x4E>(v, v));
  return fmin(v, dpp_d<0x141>(v, v));
}

// Sum over the wave; every lane gets it.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = group8_sum(v);
  v += dpp_d<0x140>(v, 0.0);          // rows of 16
  v += dpp_d<0x142, 0xA>(v, 0.0);     // rows 1 and 3 add lane 15 of the row before
  v += dpp_d<0x143, 0xC>(v, 0.0);     // rows 2 and 3 add lane 31
  return readlane_d(v, 63);
}

__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_d<0xB1>(v, v));
  v = fmax(v, dpp_d<0x4E>(v, v));
  v = fmax(v, dpp_d<0x141>(v, v));
  v = fmax(v, dpp_d<0x140>(v, v));
  v = fmax(v, dpp_d<0x142, 0xA>(v, v));
  v = fmax(v, dpp_d<0x143, 0xC>(v, v));
  return readlane_d(v, 63);
}

__device__ __forceinline__ double wave_min_dpp(double v) {
  v = fmin(v, dpp_d<0xB1>(v, v));
  v = fmin(v, dpp_d<0x4E>(v, v));
  v = fmin(v, dpp_d<0x141>(v, v));
  v = fmin(v, dpp_d<0x140>(v, v));
  v = fmin(v, dpp_d<0x142, 0xA>(v, v));
  v = fmin(v, dpp_d<0x143, 0xC>(v, v));
  return readlane_d(v, 63);
}

}  // namespace dev
}  // namespace tl
