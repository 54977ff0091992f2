// separable.h -- pieces shared by the separable-profile kernels that hold a
// spot's pixels in the registers of a lane group (the narrow kernel and the
// lane-owned kernel): row-factor broadcasts, pixel conversion and the error
// bound of the closed-form chi^2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "lanegroup.h"

namespace sf {
namespace sep {

// Row factor of row r (held by in-group lane r % L as its own[r / L]) on every
// lane of the group.
template <int L, int CPL, int R>
__device__ __forceinline__ double row_factor(const double (&own)[CPL]) {
  return lg::gbcast<L, R % L>(own[R / L]);
}

// f(r, factor of row r) for r = 0 .. HM - 1, in order.
template <int L, int CPL, int HM, int R = 0, typename F>
__device__ __forceinline__ void for_rows(const double (&own)[CPL], F&& f) {
  if constexpr (R < HM) {
    f(R, row_factor<L, CPL, R>(own));
    for_rows<L, CPL, HM, R + 1>(own, f);
  }
}

// Bound on the gap between chi^2 from the closed form and chi^2 summed over
// the pixels, in units of 2^-53 ((w + h) / 2 chi^2 + (2|a| (N FG + F G) +
// a^2 (N FF + F^2)) / N): the first-order rounding of the closed form's terms
// (the cancellations in N FG - F G and in D) plus the direct sum's own
// (sqrt(N) <= (w + h) / 2).  The largest gap measured over every workload,
// in double precision on the host, was 26 units.
constexpr double kChiGapUnits = 256.0;

// Pixel value of a stored 32-bit pattern: a 16-bit count, or a float.
template <int DT>
__device__ __forceinline__ double pixel(uint32_t v) {
  if constexpr (DT == SPOTFIT_U16)
    return double(v);
  else
    return double(__uint_as_float(v));
}

// Orders this wavefront's LDS writes before its later LDS reads (a workgroup
// is one wavefront).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

}  // namespace sep
}  // namespace sf
