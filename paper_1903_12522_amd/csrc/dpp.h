// Cross-lane neighbours through DPP wavefront shifts (an operand modifier of a VALU move, no LDS
// round trip): wave_shr:1 hands every lane the value of the lane below it, wave_shl:1 the value of
// the lane above it.  Lanes at the wavefront's ends receive 0; callers supply those lanes'
// neighbours themselves.  Every lane of the wavefront must execute the shift.
#pragma once
#include <hip/hip_runtime.h>

namespace cmcg {

// (bound_ctrl set: a lane with no source lane reads 0 in hardware, so the shift needs no zeroed
// old value, which the compiler otherwise materialises with an extra move per 32-bit shift)
__device__ __forceinline__ int dpp_shr1(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_shl1(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float lane_from_left(float x) {
  return __int_as_float(dpp_shr1(__float_as_int(x)));
}
__device__ __forceinline__ float lane_from_right(float x) {
  return __int_as_float(dpp_shl1(__float_as_int(x)));
}
__device__ __forceinline__ double lane_from_left(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)dpp_shr1((int)(unsigned)(b & 0xffffffffull));
  const unsigned hi = (unsigned)dpp_shr1((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double lane_from_right(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)dpp_shl1((int)(unsigned)(b & 0xffffffffull));
  const unsigned hi = (unsigned)dpp_shl1((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

}  // namespace cmcg
