// Cross-lane exchange within a 64-lane wavefront without the LDS crossbar
// (internal to relpic).  xor_lane<BIT>(v) returns v of lane (lane ^ BIT):
// DPP quad permutes, row shifts and the 8-lane row rotate inside each 16-lane
// row, and the gfx950 permlane swaps across rows (16) and halves (32).  All
// are VALU operations, so a chain of exchanges (a butterfly reduction) does
// not wait on the LDS pipeline as ds_bpermute does.
#pragma once

#include <hip/hip_runtime.h>

namespace relpic {

template <int BIT>
__device__ __forceinline__ int xor_lane(int v) {
  static_assert(BIT == 1 || BIT == 2 || BIT == 4 || BIT == 8 || BIT == 16 || BIT == 32, "power of two below 64");
  if constexpr (BIT == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (BIT == 2) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (BIT == 4) {
    // lanes 0-3 and 8-11 of each row read 4 lanes up (row_shl:4, banks 0 and
    // 2), lanes 4-7 and 12-15 read 4 lanes down (row_shr:4, banks 1 and 3)
    const int t = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xF, 0x5, false);
    return __builtin_amdgcn_update_dpp(t, v, 0x114, 0xF, 0xA, false);
  } else if constexpr (BIT == 8) {
    return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (BIT == 16) {
    // r[0]: rows (0, 0, 2, 2) of v, r[1]: rows (1, 1, 3, 3)
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? (int)r[0] : (int)r[1];
  } else {
    // r[0]: the low half of v in both halves, r[1]: the high half
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? (int)r[0] : (int)r[1];
  }
}

template <int BIT>
__device__ __forceinline__ float xor_lane(float v) {
  return __int_as_float(xor_lane<BIT>(__float_as_int(v)));
}

template <int BIT>
__device__ __forceinline__ double xor_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_lane<BIT>((int)(b & 0xffffffffLL)), hi = xor_lane<BIT>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// v of lane 7 - k within each aligned group of 8 lanes (lane = 8 j + k): the
// DPP row half-mirror
__device__ __forceinline__ float mirror8(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
}

__device__ __forceinline__ double mirror8(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x141, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x141, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Swap across rows (BIT 16) or halves (BIT 32): afterwards the lanes with the
// bit clear hold (a, a of lane ^ BIT) and the lanes with it set hold
// (b of lane ^ BIT, b), as (a, b).  Summing the pair gives the lane's share
// of a recursive-halving step that keeps a in the lower and b in the upper
// lanes.
template <int BIT>
__device__ __forceinline__ void swap_lanes(int &a, int &b) {
  static_assert(BIT == 16 || BIT == 32, "row or half swap");
  if constexpr (BIT == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = (int)r[0];
    b = (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = (int)r[0];
    b = (int)r[1];
  }
}

template <int BIT>
__device__ __forceinline__ void swap_lanes(float &a, float &b) {
  int x = __float_as_int(a), y = __float_as_int(b);
  swap_lanes<BIT>(x, y);
  a = __int_as_float(x);
  b = __int_as_float(y);
}

template <int BIT>
__device__ __forceinline__ void swap_lanes(double &a, double &b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  int xl = (int)(x & 0xffffffffLL), xh = (int)(x >> 32), yl = (int)(y & 0xffffffffLL), yh = (int)(y >> 32);
  swap_lanes<BIT>(xl, yl);
  swap_lanes<BIT>(xh, yh);
  a = __longlong_as_double(((long long)xh << 32) | (long long)(unsigned)xl);
  b = __longlong_as_double(((long long)yh << 32) | (long long)(unsigned)yl);
}

}  // namespace relpic
