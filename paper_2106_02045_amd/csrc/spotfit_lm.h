// spotfit_lm.h -- per-spot scalar steps of the Levenberg-Marquardt loop shared
// by the separable kernels: loop modes, limit() clamps, 10^k damping, the
// refined reciprocal and the damped 4x4 normal-equation solve (Eq. 14).
#pragma once
#include <hip/hip_runtime.h>

namespace sf {
namespace lm {

// What the next evaluation of a spot is: its start point, the first trial of
// an iteration, or a retry with more damping.
enum Mode : int { kNew = 0, kTrialFirst = 1, kTrialRetry = 2 };

__device__ __forceinline__ double clampn(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double pow10i(int k) {
  double t = 1.0;
  const int m = k < 0 ? -k : k;
  for (int i = 0; i < m; ++i) t *= 10.0;
  return k < 0 ? 1.0 / t : t;
}

// 1/x from the hardware reciprocal refined by two Newton steps (~1 ulp).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Solve (A + lam diag A) d = bv for the 4x4 symmetric A (upper triangle in
// A[10]: 00 01 02 03 11 12 13 22 23 33) by an LDL^T factorisation; NaN when a
// pivot is not positive (the matrix is not positive definite).
__device__ __forceinline__ void solve4(const double* A, const double* bv, double lam, double* d) {
  const double m00 = A[0] + lam * A[0], m11 = A[4] + lam * A[4];
  const double m22 = A[7] + lam * A[7], m33 = A[9] + lam * A[9];
  const double d0 = m00;
  bool ok = d0 > 0.0;
  const double i0 = rcp_nr(d0);
  const double l10 = A[1] * i0, l20 = A[2] * i0, l30 = A[3] * i0;
  const double d1 = m11 - l10 * l10 * d0;
  ok = ok && d1 > 0.0;
  const double i1 = rcp_nr(d1);
  const double l21 = (A[5] - l20 * l10 * d0) * i1;
  const double l31 = (A[6] - l30 * l10 * d0) * i1;
  const double d2 = m22 - l20 * l20 * d0 - l21 * l21 * d1;
  ok = ok && d2 > 0.0;
  const double i2 = rcp_nr(d2);
  const double l32 = (A[8] - l30 * l20 * d0 - l31 * l21 * d1) * i2;
  const double d3 = m33 - l30 * l30 * d0 - l31 * l31 * d1 - l32 * l32 * d2;
  ok = ok && d3 > 0.0;
  const double i3 = rcp_nr(d3);
  const double z0 = bv[0];
  const double z1 = bv[1] - l10 * z0;
  const double z2 = bv[2] - l20 * z0 - l21 * z1;
  const double z3 = bv[3] - l30 * z0 - l31 * z1 - l32 * z2;
  const double x3 = z3 * i3;
  const double x2 = z2 * i2 - l32 * x3;
  const double x1 = z1 * i1 - l21 * x2 - l31 * x3;
  const double x0 = z0 * i0 - l10 * x1 - l20 * x2 - l30 * x3;
  ok = ok && __builtin_isfinite(x0) && __builtin_isfinite(x1) && __builtin_isfinite(x2) &&
       __builtin_isfinite(x3);
  const double nanv = __builtin_nan("");
  d[0] = ok ? x0 : nanv;
  d[1] = ok ? x1 : nanv;
  d[2] = ok ? x2 : nanv;
  d[3] = ok ? x3 : nanv;
}

// Parameter j of (x, y, sx, sy): order of its x-moment and y-moment.
//   df_x = dx/sx^2 f, df_y = dy/sy^2 f, df_sx = dx^2/sx^3 f, df_sy = dy^2/sy^3 f
__device__ __forceinline__ int ox_of(int j) { return j == 0 ? 1 : j == 2 ? 2 : 0; }
__device__ __forceinline__ int oy_of(int j) { return j == 1 ? 1 : j == 3 ? 2 : 0; }

// Index pairs of the upper-triangle entries t = 0..9.
__device__ __forceinline__ int tri_i(int t) { return t < 4 ? 0 : t < 7 ? 1 : t < 9 ? 2 : 3; }
__device__ __forceinline__ int tri_j(int t) {
  return t < 4 ? t : t < 7 ? t - 3 : t < 9 ? t - 5 : 3;
}

}  // namespace lm
}  // namespace sf
