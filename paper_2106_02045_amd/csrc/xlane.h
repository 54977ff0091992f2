// xlane.h -- cross-lane sums for gfx950 wavefronts of 64 lanes.
#pragma once
#include <hip/hip_runtime.h>

namespace sf {

// ---------------------------------------------------------------------------
// Cross-lane sums over a wavefront of 64.
//
// Stage s of the tree exchanges values between lanes that differ in lane bit
// (5 - s): s = 0 v_permlane32_swap (bit 5), s = 1 v_permlane16_swap (bit 4),
// s = 2 DPP row_ror:8 (bit 3), s = 3 DPP row_half_mirror (bit 2),
// s = 4 DPP quad_perm [2,3,0,1] (bit 1), s = 5 DPP quad_perm [1,0,3,2] (bit 0).
// pair<s>(x, y) returns, on lanes whose bit is 0, x + x(partner) and, on lanes
// whose bit is 1, y + y(partner): two registers of partial sums become one.
// K values (K a power of two) are thus reduced with K-1 pair operations plus
// (6 - log2 K) single-register steps; value i ends up on every lane whose bits
// (5 - s), s < log2 K, spell the bits of i.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned as_u(float v) { return __float_as_uint(v); }
__device__ __forceinline__ float as_f(unsigned v) { return __uint_as_float(v); }

// DPP moves with bound_ctrl set: the patterns used here never read an invalid
// lane, and no "old" value has to be materialised first.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  int2 u = *reinterpret_cast<int2*>(&v);
  int2 r;
  r.x = __builtin_amdgcn_mov_dpp(u.x, CTRL, 0xF, 0xF, true);
  r.y = __builtin_amdgcn_mov_dpp(u.y, CTRL, 0xF, 0xF, true);
  return *reinterpret_cast<double*>(&r);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <int S>
struct Stage {
  static constexpr int ctrl = S == 2 ? 0x128 : S == 3 ? 0x141 : S == 4 ? 0x4E : 0xB1;
  static constexpr int bit = 5 - S;
};

template <int S>
__device__ __forceinline__ float pair(float x, float y) {
  if constexpr (S == 0) {
    auto r = __builtin_amdgcn_permlane32_swap(as_u(x), as_u(y), false, false);
    return as_f(r[0]) + as_f(r[1]);
  } else if constexpr (S == 1) {
    auto r = __builtin_amdgcn_permlane16_swap(as_u(x), as_u(y), false, false);
    return as_f(r[0]) + as_f(r[1]);
  } else {
    const bool hi = (lane_id() >> Stage<S>::bit) & 1;
    const float keep = hi ? y : x;
    const float give = hi ? x : y;
    return keep + dpp_mov<Stage<S>::ctrl>(give);
  }
}

template <int S>
__device__ __forceinline__ double pair(double x, double y) {
  if constexpr (S == 0 || S == 1) {
    int2 ux = *reinterpret_cast<int2*>(&x);
    int2 uy = *reinterpret_cast<int2*>(&y);
    int2 a, b;
    if constexpr (S == 0) {
      auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ux.x, (unsigned)uy.x, false, false);
      auto hi = __builtin_amdgcn_permlane32_swap((unsigned)ux.y, (unsigned)uy.y, false, false);
      a = make_int2((int)lo[0], (int)hi[0]);
      b = make_int2((int)lo[1], (int)hi[1]);
    } else {
      auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ux.x, (unsigned)uy.x, false, false);
      auto hi = __builtin_amdgcn_permlane16_swap((unsigned)ux.y, (unsigned)uy.y, false, false);
      a = make_int2((int)lo[0], (int)hi[0]);
      b = make_int2((int)lo[1], (int)hi[1]);
    }
    return *reinterpret_cast<double*>(&a) + *reinterpret_cast<double*>(&b);
  } else {
    const bool hi = (lane_id() >> Stage<S>::bit) & 1;
    const double keep = hi ? y : x;
    const double give = hi ? x : y;
    return keep + dpp_mov<Stage<S>::ctrl>(give);
  }
}

template <int S, typename T>
__device__ __forceinline__ void finish(T& v) {
  if constexpr (S < 6) {
    v = pair<S>(v, v);
    finish<S + 1>(v);
  }
}

template <int S, int K, typename T>
__device__ __forceinline__ void halve(T* v) {
  if constexpr (K > 1) {
#pragma unroll
    for (int i = 0; i < K / 2; ++i) v[i] = pair<S>(v[2 * i], v[2 * i + 1]);
    halve<S + 1, K / 2>(v);
  } else {
    finish<S>(v[0]);
  }
}

template <int K>
struct Log2 {
  static constexpr int v = K <= 1 ? 0 : 1 + Log2<(K / 2)>::v;
};
template <>
struct Log2<1> {
  static constexpr int v = 0;
};

template <int K>
__host__ __device__ constexpr int lane_of(int i) {
  int l = 0;
  for (int s = 0; s < Log2<K>::v; ++s) l |= ((i >> s) & 1) << (5 - s);
  return l;
}

__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double bcast(double v, int lane) {
  int2 u = *reinterpret_cast<int2*>(&v);
  int2 r = make_int2(__builtin_amdgcn_readlane(u.x, lane), __builtin_amdgcn_readlane(u.y, lane));
  return *reinterpret_cast<double*>(&r);
}

// Sum each of the first M entries of v[K] over the wavefront; results are
// wave-uniform.  Entries M..K-1 are scratch.
template <int K, int M, typename T>
__device__ __forceinline__ void wave_sums(T (&v)[K], T (&out)[M]) {
  static_assert((K & (K - 1)) == 0 && K >= M && K <= 64, "K must be a power of two");
  halve<0, K>(v);
#pragma unroll
  for (int i = 0; i < M; ++i) out[i] = bcast(v[0], lane_of<K>(i));
}

template <typename T>
__device__ __forceinline__ T wave_sum1(T v) {
  finish<0>(v);
  return bcast(v, 0);
}


// Group reductions: a group is L consecutive lanes (L = 8, 16, 32 or 64, aligned).
// Stages 6 - log2(L) .. 5 exchange only inside a group.
template <int L>
struct GroupLog {
  static constexpr int m = L == 64 ? 6 : L == 32 ? 5 : L == 16 ? 4 : L == 8 ? 3 : L == 4 ? 2 : -1;
  static_assert(m > 0, "group size must be 4, 8, 16, 32 or 64");
};

template <int S, int K, typename T>
__device__ __forceinline__ void halve_from(T* v) {
  if constexpr (K > 1 && S < 6) {
#pragma unroll
    for (int i = 0; i < K / 2; ++i) v[i] = pair<S>(v[2 * i], v[2 * i + 1]);
    halve_from<S + 1, K / 2>(v);
  } else if constexpr (S < 6) {
    finish<S>(v[0]);
  }
}

// Value index held by register i of a lane after group_halve<L, K>:
// for K >= L, register i of in-group lane l holds value L*i + rev(l) (rev =
// bit reversal over log2 L bits); for K < L, register 0 holds value
// rev(l) >> (log2 L - log2 K), totalled over the whole group.
__device__ __forceinline__ int bitrev_bits(int l, int bits) {
  int r = 0;
  for (int t = 0; t < bits; ++t) r |= ((l >> (bits - 1 - t)) & 1) << t;
  return r;
}

template <int L, int K, typename T>
__device__ __forceinline__ void group_halve(T (&v)[K]) {
  static_assert((K & (K - 1)) == 0, "K must be a power of two");
  halve_from<6 - GroupLog<L>::m, K>(v);
}

}  // namespace sf
