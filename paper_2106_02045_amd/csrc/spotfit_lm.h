// spotfit_lm.h -- per-spot scalar steps of the Levenberg-Marquardt loop shared
// by the separable kernels: loop modes, limit() clamps, 10^k damping, the
// refined reciprocal and the damped 4x4 normal-equation solve (Eq. 14).
#pragma once
#include <hip/hip_runtime.h>

namespace sf {
namespace lm {

// What the next evaluation of a spot is: its start point, the first trial of
// an iteration, or a retry with more damping.
enum Mode : int { kNew = 0, kTrialFirst = 1, kTrialRetry = 2,
                  // re-evaluations with a directly summed chi^2 before a close decision
                  kRecheckBest = 3, kRecheckCand = 4 };

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

// a * b + c with c taken from a scalar register pair: keeps polynomial
// constants out of vector registers (and out of the per-step copies a
// vector-register accumulator would need).
__device__ __forceinline__ double fma_s(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// e^x for x <= 0 (the argument of a Gaussian factor), within ~1 ulp:
// x = n ln2 + r with |r| <= ln2 / 2 (Cody-Waite reduction with ln 2 split into
// its double value and the double nearest the remainder, each step one fused
// multiply-add), e^r by its Taylor series to degree 13 (truncation below 5e-18
// relative on that interval), scaled by 2^n.  Underflows to 0 for x below
// about -745; NaN stays NaN.
__device__ __forceinline__ double exp_neg(double x) {
  constexpr double kLog2e = 1.4426950408889634;
  constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;   // ln 2 rounded to double
  constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;  // ln 2 - kLn2Hi
  const double n = __builtin_rint(x * kLog2e);
  double r = __builtin_fma(-n, kLn2Hi, x);
  r = __builtin_fma(-n, kLn2Lo, r);
  // Taylor coefficients 1/k!, k = 13 .. 2, in Horner order
  double p = 1.0 / 6227020800.0;                 // 1/13!
  p = fma_s(p, r, 1.0 / 479001600.0);            // 1/12!
  p = fma_s(p, r, 1.0 / 39916800.0);             // 1/11!
  p = fma_s(p, r, 1.0 / 3628800.0);              // 1/10!
  p = fma_s(p, r, 1.0 / 362880.0);               // 1/9!
  p = fma_s(p, r, 1.0 / 40320.0);                // 1/8!
  p = fma_s(p, r, 1.0 / 5040.0);                 // 1/7!
  p = fma_s(p, r, 1.0 / 720.0);                  // 1/6!
  p = fma_s(p, r, 1.0 / 120.0);                  // 1/5!
  p = fma_s(p, r, 1.0 / 24.0);                   // 1/4!
  p = fma_s(p, r, 1.0 / 6.0);                    // 1/3!
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return __builtin_ldexp(p, (int)n);
}

// e^x[i] for N independent arguments x[i] <= 0 (each as exp_neg), with the
// steps of the N evaluations interleaved: the multiply-adds of different
// arguments are independent, so N of them are in flight together instead of
// one dependent chain of 13 after another.
template <int N>
__device__ __forceinline__ void exp_neg_n(const double (&x)[N], double (&y)[N]) {
  constexpr double kLog2e = 1.4426950408889634;
  constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;
  constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;
  constexpr double kC[11] = {1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0,
                             1.0 / 362880.0,    1.0 / 40320.0,    1.0 / 5040.0,
                             1.0 / 720.0,       1.0 / 120.0,      1.0 / 24.0,
                             1.0 / 6.0,         0.5};  // 1/k!, k = 12 .. 2
  double n[N], r[N], p[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    n[i] = __builtin_rint(x[i] * kLog2e);
    r[i] = __builtin_fma(-n[i], kLn2Hi, x[i]);
    r[i] = __builtin_fma(-n[i], kLn2Lo, r[i]);
    p[i] = 1.0 / 6227020800.0;  // 1/13!
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) {
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = fma_s(p[i], r[i], kC[k]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    p[i] = __builtin_fma(p[i], r[i], kC[10]);
    p[i] = __builtin_fma(p[i], r[i], 1.0);
    p[i] = __builtin_fma(p[i], r[i], 1.0);
    y[i] = __builtin_ldexp(p[i], (int)n[i]);
  }
}

}  // namespace lm
}  // namespace sf
