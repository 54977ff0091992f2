// separable.h -- pieces shared by the separable-profile kernels that hold a
// spot's pixels in the registers of a lane group (the narrow kernel and the
// lane-owned kernel): row-factor broadcasts, pixel conversion and the error
// bound of the closed-form chi^2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "lanegroup.h"
#include "spotfit_lm.h"

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

// Eq. 6 from the group sums Sx = sum ex, Sxx = sum ex^2, Sy, Syy, FG = **G**
// and G = sum g: F = Sx Sy, FF = Sxx Syy (**F**), D = N FF - F^2,
// a = (N FG - F G) / D, b = (G FF - F FG) / D.  Each difference of products is
// one fused multiply-add of the first product with the rounded second, written
// out so that every kernel using it rounds alike.
struct Amplitudes {
  double F, FF, D, iD, a, b;
};

__device__ __forceinline__ Amplitudes amplitudes(double Nn, double Sx, double Sxx, double Sy, double Syy,
                                                 double FG, double G) {
  Amplitudes r;
  r.F = Sx * Sy;
  r.FF = Sxx * Syy;
  r.D = __builtin_fma(Nn, r.FF, -(r.F * r.F));
  r.iD = lm::rcp_nr(r.D);
  r.a = __builtin_fma(Nn, FG, -(r.F * G)) * r.iD;
  r.b = __builtin_fma(G, r.FF, -(r.F * FG)) * r.iD;
  return r;
}

// chi^2 of 16-bit data at the amplitudes of Eq. 6 without a second pixel pass:
// with sum r = sum f r = 0 (Eq. 4), chi^2 = sum (g - mean g)^2 - a^2 sum
// (f - mean f)^2 = (V - a^2 D) / N, V = N sum g^2 - G^2 exact (clamped at 0);
// err: the bound on its gap to chi^2 summed over the pixels (kChiGapUnits).
// Bright spots cancel the most: up to 3e-11 of chi^2 measured.
__device__ __forceinline__ void chi_closed(double Vs, const Amplitudes& am, double Nn, double FG, double G,
                                           int w, int h, double& chi, double& err) {
  const double iNn = lm::rcp_nr(Nn);
  const double c2 = __builtin_fma(-(am.a * am.a), am.D, Vs) * iNn;
  chi = c2 > 0.0 ? c2 : 0.0;
  const double s1 = __builtin_fma(Nn, FG, am.F * G);
  const double s2 = __builtin_fma(Nn, am.FF, am.F * am.F);
  const double t = __builtin_fma(2.0 * fabs(am.a), s1, am.a * am.a * s2);
  err = kChiGapUnits * 0x1p-53 * __builtin_fma(0.5 * double(w + h), chi, t * iNn);
}

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
