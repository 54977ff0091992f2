// lanegroup.h -- operations inside a group of L consecutive lanes (L = 1, 2, 4,
// 8 or 16, aligned; the totals and minima also L = 32) of a gfx950 wavefront,
// by DPP, ds_swizzle or permlane16_swap.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xlane.h"

namespace sf {
namespace lg {

// Both halves of a pair of 16-lane rows (lanes l and l ^ 16): permlane16_swap
// of a value with itself gives the even row's value in [0] and the odd row's
// in [1] on every lane of the pair.
__device__ __forceinline__ void row_pair(uint32_t v, uint32_t& even, uint32_t& odd) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  even = r[0];
  odd = r[1];
}

// Total over the group: butterfly over lane bits 0 (quad_perm [1,0,3,2]), 1
// (quad_perm [2,3,0,1]), 2 (row_half_mirror), 3 (row_mirror) and 4 (pairs of
// rows).  The two partners of a step add the same two numbers, so every lane of
// the group holds bitwise the same total.
template <int L>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (L >= 2) v += dpp_mov<0xB1>(v);
  if constexpr (L >= 4) v += dpp_mov<0x4E>(v);
  if constexpr (L >= 8) v += dpp_mov<0x141>(v);
  if constexpr (L >= 16) v += dpp_mov<0x140>(v);
  if constexpr (L >= 32) v = pair<1>(v, v);
  return v;
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int L>
__device__ __forceinline__ int gsum_i(int v) {
  if constexpr (L >= 2) v += dpp_i<0xB1>(v);
  if constexpr (L >= 4) v += dpp_i<0x4E>(v);
  if constexpr (L >= 8) v += dpp_i<0x141>(v);
  if constexpr (L >= 16) v += dpp_i<0x140>(v);
  if constexpr (L >= 32) {
    uint32_t e, o;
    row_pair((uint32_t)v, e, o);
    v = (int)e + (int)o;
  }
  return v;
}

template <int L>
__device__ __forceinline__ uint32_t gmin_u(uint32_t v) {
  uint32_t t;
  if constexpr (L >= 2) { t = (uint32_t)dpp_i<0xB1>((int)v); v = t < v ? t : v; }
  if constexpr (L >= 4) { t = (uint32_t)dpp_i<0x4E>((int)v); v = t < v ? t : v; }
  if constexpr (L >= 8) { t = (uint32_t)dpp_i<0x141>((int)v); v = t < v ? t : v; }
  if constexpr (L >= 16) { t = (uint32_t)dpp_i<0x140>((int)v); v = t < v ? t : v; }
  if constexpr (L >= 32) {
    uint32_t e, o;
    row_pair(v, e, o);
    v = e < o ? e : o;
  }
  return v;
}

// Value of in-group lane Q on every lane of the group.
template <int L, int Q>
__device__ __forceinline__ int gbcast_i(int v) {
  if constexpr (L == 1) {
    return v;
  } else if constexpr (L == 2) {
    return __builtin_amdgcn_mov_dpp(v, Q == 0 ? 0xA0 : 0xF5, 0xF, 0xF, true);
  } else if constexpr (L == 4) {
    return __builtin_amdgcn_mov_dpp(v, Q * 0x55, 0xF, 0xF, true);
  } else {
    // ds_swizzle bit-mask mode inside 32 lanes: lane' = (lane & and) | Q
    constexpr int andm = L == 8 ? 0x18 : 0x10;
    return __builtin_amdgcn_ds_swizzle(v, andm | (Q << 5));
  }
}

template <int L, int Q>
__device__ __forceinline__ double gbcast(double v) {
  // a 16-lane group is a DPP row: one 64-bit move broadcasts its lane Q
  // (row_newbcast, the one DPP control of gfx950's 64-bit moves)
  if constexpr (L == 16) return __builtin_amdgcn_update_dpp(0.0, v, 0x150 | Q, 0xF, 0xF, false);
  int2 u = *reinterpret_cast<int2*>(&v);
  int2 r = make_int2(gbcast_i<L, Q>(u.x), gbcast_i<L, Q>(u.y));
  return *reinterpret_cast<double*>(&r);
}

}  // namespace lg
}  // namespace sf
