// spotfit_kernels.hip -- gfx950 kernels of the batched implicit-amplitude
// Levenberg-Marquardt Gaussian-spot fit (Leutenegger & Weber).
//
// Mapping (one wavefront per spot): the 64 lanes of a wave own the pixels of one
// spot, PPL pixels per lane (pixel k = j*64 + lane, j < PPL).  Pixel values and
// coordinates stay in registers for the whole fit; every evaluation of the model
// is a pass over those registers followed by cross-lane sums.  The per-spot
// scalars (parameters, amplitudes, the 3x3/4x4 normal matrix, damping, stop
// tests) are wave-uniform.  The paper's design gives one thread per pixel and
// sums through warp shuffles and shared memory; here a 64-wide wavefront sums
// many values at once with a recursive-halving tree built from gfx950's
// v_permlane32_swap / v_permlane16_swap and DPP row operations, with no LDS.
//
// One evaluation at the parameters p ("trial" evaluation, Eqs. 2-6):
//   f_k = exp(-(x_k-x)^2/(2 sx^2) - (y_k-y)^2/(2 sy^2))       (Eq. 10; sx = sy sym.)
//   F, FF = sum f^2, FG = sum f g -> D = N FF - F^2,
//   alpha = (N FG - F G)/D, beta = (G FF - F FG)/D             (Eqs. 5-6)
//   chi^2 = sum (alpha f + beta - g)^2                            (Eq. 2)
// The derivative pass at an accepted point adds (Eqs. 7-9, 11):
//   dF_j, dFF_j = 2 sum f df_j, dFG_j = sum g df_j, gamma_j, d alpha_j, d beta_j,
//   J_kj = d alpha_j f_k + alpha df_kj + d beta_j  (= d r_k / d p_j),
//   A = J^T J, b = -J^T r
// and the damped step solves (A + lambda diag A) delta = b (Eq. 14) by Cholesky.
//
// Precision (template parameter S = scalar type):
//   S = double  ("mixed"): parameters, pixel offsets and the exponent in double,
//               exp and derivative terms in float, per-lane float partial sums
//               combined by a pairwise tree, D / alpha / beta / derivatives of
//               the amplitudes / LM solve / residuals and the chi^2 sum in double.
//   S = float   ("fp32"): everything in single precision, the paper's arithmetic.
//   S = double, COMP ("comp"): as "mixed", but every per-lane sum of the
//               evaluations (F, FF, FG and the derivative and normal-equation
//               sums) is a compensated single-precision sum -- each product's
//               rounding error recovered with an fma and each addition's with
//               TwoSum, carried in a second float -- and the lane totals
//               (sum + error, exact in double) are combined in double.  The
//               profile and the per-pixel products stay single precision.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "xlane.h"

namespace sf {

// ---------------------------------------------------------------------------
// Per-spot fit
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ bool finite_s(S v) {
  return __builtin_isfinite(v);
}
__device__ __forceinline__ float fma_s(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_s(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float sqrt_s(float v) { return __builtin_sqrtf(v); }
__device__ __forceinline__ double sqrt_s(double v) { return __builtin_sqrt(v); }
__device__ __forceinline__ float fabs_s(float v) { return __builtin_fabsf(v); }
__device__ __forceinline__ double fabs_s(double v) { return __builtin_fabs(v); }

template <typename S>
__device__ __forceinline__ S clamp_nan(S v, S lo, S hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// 10^k from its definition: exact products of ten, reciprocal for k < 0.
template <typename S>
__device__ __forceinline__ S pow10_s(int k) {
  S t = S(1);
  const int m = k < 0 ? -k : k;
  for (int i = 0; i < m; ++i) t *= S(10);
  return k < 0 ? S(1) / t : t;
}

// Cholesky solve of (A + lam diag A) d = b for n = NP; NaN on failure.
template <int NP, typename S>
__device__ __forceinline__ void damped_solve(const S (&A)[NP][NP], const S (&b)[NP], S lam,
                                             S (&d)[NP]) {
  S L[NP][NP];
  S y[NP];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    S s = A[j][j] + lam * A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    ok = ok && (s > S(0)) && finite_s(s);
    const S ljj = sqrt_s(s);  // NaN if s <= 0: caught by ok
    L[j][j] = ljj;
#pragma unroll
    for (int i = j + 1; i < NP; ++i) {
      S t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / ljj;
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    S t = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
    y[i] = t / L[i][i];
  }
#pragma unroll
  for (int i = NP - 1; i >= 0; --i) {
    S t = y[i];
#pragma unroll
    for (int k = i + 1; k < NP; ++k) t -= L[k][i] * d[k];
    d[i] = t / L[i][i];
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) ok = ok && finite_s(d[i]);
  if (!ok) {
#pragma unroll
    for (int i = 0; i < NP; ++i) d[i] = __builtin_nan("");
  }
}

// A single-precision sum with its running rounding error: error-free
// transformations of the addition (Knuth's TwoSum) and of the product (by fma),
// as in the compensated dot product of Ogita, Rump and Oishi (SIAM J. Sci.
// Comput. 26, 2005).  value() = s + c in double.
struct CSum {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float x) {
#pragma clang fp contract(off)
    const float t = s + x;
    const float z = t - s;
    c += (s - (t - z)) + (x - z);
    s = t;
  }
  __device__ __forceinline__ void add_prod(float a, float b) {
#pragma clang fp contract(off)
    const float p = a * b;
    const float pe = __builtin_fmaf(a, b, -p);  // a * b - p, exactly
    add(p);
    c += pe;
  }
  __device__ __forceinline__ double value() const { return double(s) + double(c); }
};

constexpr float kOffGrid = 4096.0f;  // coordinate of padding lanes: exp(-huge) = 0

template <int PPL>
struct Pixels {
  float g[PPL];   // pixel values (0 on padding)
  float xs[PPL];  // column of the pixel (kOffGrid on padding)
  float ys[PPL];  // row of the pixel
  float m[PPL];   // 1 on pixels of the spot, 0 on padding
};

// Uniform amplitude state at one parameter point.
template <typename S>
struct AmpState {
  S F, FF, FG, D, a, b, chi;
};

template <int NP, typename S>
struct Geo {
  S p[NP];
};

template <int MODEL>
struct Np {
  static constexpr int v = MODEL == SPOTFIT_SYM ? 3 : 4;
};

// Profile exponent scale: exp(-q/2) = exp2(q * kNegHalfLog2e).
constexpr double kNegHalfLog2e = -0.72134752044448170368;  // -0.5 / ln 2

// Trial evaluation at p: fills f[], returns amplitudes and chi^2 (NaN if D <= 0).
template <int PPL, int MODEL, typename S, bool COMP>
__device__ __forceinline__ AmpState<S> eval_trial(const Pixels<PPL>& px, float (&f)[PPL],
                                                  const S (&p)[Np<MODEL>::v], int N, S G) {
  const S isx2 = S(1) / (p[2] * p[2]);
  const S isy2 = (MODEL == SPOTFIT_SYM) ? isx2 : S(1) / (p[3] * p[3]);
  const S c = S(kNegHalfLog2e);
  AmpState<S> st;
  if constexpr (COMP) {
    CSum cs[3];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const S dx = S(px.xs[j]) - p[0];
      const S dy = S(px.ys[j]) - p[1];
      const S q = dx * dx * isx2 + dy * dy * isy2;
      const float e = __builtin_amdgcn_exp2f(float(q * c));
      f[j] = e;
      cs[0].add(e);
      cs[1].add_prod(e, e);
      cs[2].add_prod(e, px.g[j]);
    }
    double acc[4] = {cs[0].value(), cs[1].value(), cs[2].value(), 0.0};
    double s3[3];
    wave_sums<4, 3>(acc, s3);
    st.F = s3[0];
    st.FF = s3[1];
    st.FG = s3[2];
  } else {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const S dx = S(px.xs[j]) - p[0];
      const S dy = S(px.ys[j]) - p[1];
      const S q = dx * dx * isx2 + dy * dy * isy2;
      const float e = __builtin_amdgcn_exp2f(float(q * c));
      f[j] = e;
      acc[0] += e;
      acc[1] = __builtin_fmaf(e, e, acc[1]);
      acc[2] = __builtin_fmaf(e, px.g[j], acc[2]);
    }
    float s3[3];
    wave_sums<4, 3>(acc, s3);
    st.F = S(s3[0]);
    st.FF = S(s3[1]);
    st.FG = S(s3[2]);
  }
  const S Nn = S(N);
  st.D = Nn * st.FF - st.F * st.F;
  const S nanv = S(__builtin_nan(""));
  if (!(st.D > S(0)) || !finite_s(st.D)) {
    st.a = st.b = st.chi = nanv;
    return st;
  }
  st.a = (Nn * st.FG - st.F * G) / st.D;
  st.b = (G * st.FF - st.F * st.FG) / st.D;
  S chi = S(0);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    // r = alpha f + beta - g, padding lanes give exactly 0 (f = 0, m = 0, g = 0)
    const S r = fma_s(st.a, S(f[j]), fma_s(st.b, S(px.m[j]), -S(px.g[j])));
    chi = fma_s(r, r, chi);
  }
  st.chi = wave_sum1(chi);
  if (!finite_s(st.chi) || !finite_s(st.a) || !finite_s(st.b)) st.chi = nanv;
  return st;
}

// Derivatives of the profile at pixel j (Eq. 11, and its elliptical analogue).
template <int MODEL>
__device__ __forceinline__ void dprofile(float fj, float dx, float dy, float isx, float isx2,
                                         float isy, float isy2, float (&df)[Np<MODEL>::v]) {
  if constexpr (MODEL == SPOTFIT_SYM) {
    const float t = fj * isx2;
    df[0] = dx * t;
    df[1] = dy * t;
    df[2] = __builtin_fmaf(dx, dx, dy * dy) * t * isx;
  } else {
    const float tx = fj * isx2;
    const float ty = fj * isy2;
    df[0] = dx * tx;
    df[1] = dy * ty;
    df[2] = dx * dx * tx * isx;
    df[3] = dy * dy * ty * isy;
  }
}

template <int N>
struct Pow2Ceil {
  static constexpr int v = N <= 1 ? 1 : N <= 2 ? 2 : N <= 4 ? 4 : N <= 8 ? 8 : N <= 16 ? 16 : 32;
};

// Derivative evaluation at p (f, alpha, beta and sums of the trial evaluation at
// the same p are reused): normal matrix A and right-hand side b.
template <int PPL, int MODEL, typename S, bool COMP>
__device__ __forceinline__ void eval_grad(const Pixels<PPL>& px, const float (&f)[PPL],
                                          const S (&p)[Np<MODEL>::v], int N, S G,
                                          const AmpState<S>& st, S (&A)[Np<MODEL>::v][Np<MODEL>::v],
                                          S (&bv)[Np<MODEL>::v]) {
  constexpr int NP = Np<MODEL>::v;
  const S isx = S(1) / p[2];
  const S isy = (MODEL == SPOTFIT_SYM) ? isx : S(1) / p[3];
  const float isxf = float(isx), isyf = float(isy);
  const float isx2f = float(isx * isx), isy2f = float(isy * isy);

  // round A: dF_j, sum f df_j, dFG_j (Eq. 7)
  constexpr int KA = Pow2Ceil<3 * NP>::v;
  using SumT = typename std::conditional<COMP, double, float>::type;
  SumT sA[3 * NP];
  if constexpr (COMP) {
    CSum cs[3 * NP];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const float dx = float(S(px.xs[j]) - p[0]);
      const float dy = float(S(px.ys[j]) - p[1]);
      float df[NP];
      dprofile<MODEL>(f[j], dx, dy, isxf, isx2f, isyf, isy2f, df);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        cs[q].add(df[q]);
        cs[NP + q].add_prod(f[j], df[q]);
        cs[2 * NP + q].add_prod(px.g[j], df[q]);
      }
    }
    double acc[KA];
#pragma unroll
    for (int i = 0; i < KA; ++i) acc[i] = i < 3 * NP ? cs[i].value() : 0.0;
    wave_sums<KA, 3 * NP>(acc, sA);
  } else {
    float acc[KA];
#pragma unroll
    for (int i = 0; i < KA; ++i) acc[i] = 0.f;
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const float dx = float(S(px.xs[j]) - p[0]);
      const float dy = float(S(px.ys[j]) - p[1]);
      float df[NP];
      dprofile<MODEL>(f[j], dx, dy, isxf, isx2f, isyf, isy2f, df);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        acc[q] += df[q];
        acc[NP + q] = __builtin_fmaf(f[j], df[q], acc[NP + q]);
        acc[2 * NP + q] = __builtin_fmaf(px.g[j], df[q], acc[2 * NP + q]);
      }
    }
    wave_sums<KA, 3 * NP>(acc, sA);
  }

  // Eq. 8: derivatives of the amplitudes
  const S Nn = S(N);
  S da[NP], db[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const S dF = S(sA[q]);
    const S dFF = S(2) * S(sA[NP + q]);
    const S dFG = S(sA[2 * NP + q]);
    const S gam = Nn * dFF - S(2) * st.F * dF;
    da[q] = (Nn * dFG - G * dF - st.a * gam) / st.D;
    db[q] = (G * dFF - st.FG * dF - st.F * dFG - st.b * gam) / st.D;
  }

  // round B: J = d r / d p (Eq. 9, second factor), A = J^T J, J^T r
  constexpr int NB = NP * (NP + 1) / 2 + NP;
  constexpr int KB = Pow2Ceil<NB>::v;
  float bcc[COMP ? 1 : KB];
  CSum bcs[COMP ? NB : 1];
  if constexpr (!COMP) {
#pragma unroll
    for (int i = 0; i < KB; ++i) bcc[i] = 0.f;
  }
  const float af = float(st.a);
  float daf[NP], dbf[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    daf[q] = float(da[q]);
    dbf[q] = float(db[q]);
  }
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const float dx = float(S(px.xs[j]) - p[0]);
    const float dy = float(S(px.ys[j]) - p[1]);
    float df[NP];
    dprofile<MODEL>(f[j], dx, dy, isxf, isx2f, isyf, isy2f, df);
    const float r = float(fma_s(st.a, S(f[j]), fma_s(st.b, S(px.m[j]), -S(px.g[j]))));
    float Jk[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q)
      Jk[q] = __builtin_fmaf(daf[q], f[j], __builtin_fmaf(af, df[q], dbf[q] * px.m[j]));
    int t = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int u = q; u < NP; ++u) {
        if constexpr (COMP)
          bcs[t].add_prod(Jk[q], Jk[u]);
        else
          bcc[t] = __builtin_fmaf(Jk[q], Jk[u], bcc[t]);
        ++t;
      }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if constexpr (COMP)
        bcs[t + q].add_prod(Jk[q], r);
      else
        bcc[t + q] = __builtin_fmaf(Jk[q], r, bcc[t + q]);
    }
  }
  SumT sB[NB];
  if constexpr (COMP) {
    double acc[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) acc[i] = i < NB ? bcs[i].value() : 0.0;
    wave_sums<KB, NB>(acc, sB);
  } else {
    wave_sums<KB, NB>(bcc, sB);
  }
  int t = 0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
#pragma unroll
    for (int u = q; u < NP; ++u) {
      A[q][u] = S(sB[t]);
      A[u][q] = S(sB[t]);
      ++t;
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) bv[q] = -S(sB[t + q]);
}

template <int MODEL, typename S>
__device__ __forceinline__ void limit_p(S (&p)[Np<MODEL>::v], int w, int h, const KOpts& o) {
  const S smax = S(o.sigma_max_frac) * S(w > h ? w : h);
  p[0] = clamp_nan(p[0], S(-0.5), S(w) - S(0.5));
  p[1] = clamp_nan(p[1], S(-0.5), S(h) - S(0.5));
  p[2] = clamp_nan(p[2], S(o.sigma_min), smax);
  if constexpr (MODEL == SPOTFIT_ELL) p[3] = clamp_nan(p[3], S(o.sigma_min), smax);
}

template <int NP, typename S>
// MinStep: every |d_j| below rel times its parameter, the centre coordinates
// measured from the centre (cx, cy) of the ROI.
__device__ __forceinline__ bool all_small(const S (&d)[NP], const S (&best)[NP], S rel, S cx, S cy) {
  bool all = true;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const S lim = rel * fabs_s(best[j] - (j == 0 ? cx : j == 1 ? cy : S(0)));
    all = all && (fabs_s(d[j]) < lim);
  }
  return all;
}

struct SpotOut {
  float p[6];
  float chi2;
  int iters, status, n_grad, n_trial;
};

// The Levenberg-Marquardt loop of one spot (Fit2DGaussian pseudo-code).
template <int PPL, int MODEL, typename S, bool COMP>
__device__ SpotOut lm_fit(const Pixels<PPL>& px, int N, S G, const float* init4, int w, int h,
                          const KOpts& o) {
  constexpr int NP = Np<MODEL>::v;
  SpotOut out;
  float f[PPL];
  S p[NP], best[NP], delta[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) p[q] = S(init4[q]);

  const S T = S(o.max_error_per_px) * S(N);
  const S tau = S(o.tie_tau);
  const S min_delta = S(o.min_delta);
  const S min_step = S(o.min_step_rel);
  const S cx = S(0.5) * S(w - 1), cy = S(0.5) * S(h - 1);  // centre of the ROI
  int k = o.lambda0_exp10;
  int it = 0, status = SPOTFIT_MAX_ITER, n_grad = 0, n_trial = 0;

  // state at the current point p
  AmpState<S> cur = eval_trial<PPL, MODEL, S, COMP>(px, f, p, N, G);
  AmpState<S> keep = cur;  // state at best
  S A[NP][NP], bv[NP];

  while (it < o.max_iter) {
    ++it;
    const S chi = cur.chi;
    if (__builtin_isnan(chi)) { status = SPOTFIT_NOT_CONVERGED; break; }
    if (chi < T) { status = SPOTFIT_MAX_ERROR; break; }
    eval_grad<PPL, MODEL, S, COMP>(px, f, p, N, G, cur, A, bv);
    ++n_grad;
#pragma unroll
    for (int q = 0; q < NP; ++q) best[q] = p[q];
    keep = cur;

    damped_solve<NP, S>(A, bv, pow10_s<S>(k), delta);
#pragma unroll
    for (int q = 0; q < NP; ++q) p[q] = best[q] + delta[q];
    limit_p<MODEL, S>(p, w, h, o);
    cur = eval_trial<PPL, MODEL, S, COMP>(px, f, p, N, G);
    ++n_trial;
    if (cur.chi < chi * (S(1) - tau)) --k;  // improved: less damping

    while (!all_small<NP, S>(delta, best, min_step, cx, cy) && (chi * (S(1) + tau) < cur.chi) &&
           k < o.lambda_max_exp10) {
      ++k;  // worse: more damping, retry from best
      damped_solve<NP, S>(A, bv, pow10_s<S>(k), delta);
#pragma unroll
      for (int q = 0; q < NP; ++q) p[q] = best[q] + delta[q];
      limit_p<MODEL, S>(p, w, h, o);
      cur = eval_trial<PPL, MODEL, S, COMP>(px, f, p, N, G);
      ++n_trial;
    }
    if ((chi * (S(1) + tau) < cur.chi) || __builtin_isnan(cur.chi)) {
#pragma unroll
      for (int q = 0; q < NP; ++q) p[q] = best[q];
      cur = keep;
      status = SPOTFIT_NOT_CONVERGED;
      break;
    }
    if (cur.chi < T) { status = SPOTFIT_MAX_ERROR; break; }
    if (chi * (S(1) - min_delta) < cur.chi) { status = SPOTFIT_MIN_DELTA; break; }
    if (all_small<NP, S>(delta, best, min_step, cx, cy)) { status = SPOTFIT_MIN_STEP; break; }
  }

  out.p[0] = float(p[0]);
  out.p[1] = float(p[1]);
  out.p[2] = float(p[2]);
  out.p[3] = float(MODEL == SPOTFIT_ELL ? p[NP - 1] : p[2]);
  out.p[4] = float(cur.a);
  out.p[5] = float(cur.b);
  out.chi2 = float(cur.chi);
  out.iters = it;
  out.status = status;
  out.n_grad = n_grad;
  out.n_trial = n_trial;
  return out;
}

template <int PPL>
__device__ __forceinline__ double load_pixels(Pixels<PPL>& px, const void* data, int dtype,
                                              int64_t off, int w, int N) {
  const int lane = lane_id();
  int row = lane / w;
  int col = lane - row * w;
  const int drow = 64 / w;
  const int dcol = 64 - drow * w;
  double gsum = 0.0;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int kk = j * 64 + lane;
    const bool v = kk < N;
    float gv = 0.f;
    if (v) {
      if (dtype == SPOTFIT_U16)
        gv = float(static_cast<const uint16_t*>(data)[off + kk]);
      else
        gv = static_cast<const float*>(data)[off + kk];
    }
    px.g[j] = gv;
    px.m[j] = v ? 1.f : 0.f;
    px.xs[j] = v ? float(col) : kOffGrid;
    px.ys[j] = v ? float(row) : kOffGrid;
    gsum += double(gv);
    col += dcol;
    row += drow;
    if (col >= w) {
      col -= w;
      row += 1;
    }
  }
  return wave_sum1(gsum);
}

template <int PPL, typename S, bool COMP>
__global__ __launch_bounds__(64) void fit_wave_kernel(KArgs ka) {
  const int lane = lane_id();
  for (int64_t s = blockIdx.x; s < ka.n; s += gridDim.x) {
    const spotfit_shape_t sh = ka.sizes[s];
    const int w = sh.w, h = sh.h, model = sh.model;
    const int N = w * h;
    const float* init4 = ka.init + 4 * s;
    float i0 = init4[0], i1 = init4[1], i2 = init4[2], i3 = init4[3];
    const bool ell = model == SPOTFIT_ELL;
    bool bad = w < 3 || h < 3 || N > 64 * PPL || N > ka.opt.max_pixels ||
               w > ka.opt.max_side || h > ka.opt.max_side ||
               (model != SPOTFIT_SYM && model != SPOTFIT_ELL) || !__builtin_isfinite(i0) ||
               !__builtin_isfinite(i1) || !__builtin_isfinite(i2) || !(i2 > 0.f) ||
               (ell && (!__builtin_isfinite(i3) || !(i3 > 0.f)));
    SpotOut out;
    if (bad) {
      const float nanf = __builtin_nanf("");
      for (int q = 0; q < 6; ++q) out.p[q] = nanf;
      out.chi2 = nanf;
      out.iters = 0;
      out.status = SPOTFIT_BAD_INPUT;
      out.n_grad = out.n_trial = 0;
    } else {
      Pixels<PPL> px;
      const double G = load_pixels<PPL>(px, ka.data, ka.dtype, ka.offsets[s], w, N);
      if (!ell)
        out = lm_fit<PPL, SPOTFIT_SYM, S, COMP>(px, N, S(G), init4, w, h, ka.opt);
      else
        out = lm_fit<PPL, SPOTFIT_ELL, S, COMP>(px, N, S(G), init4, w, h, ka.opt);
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 6; ++q) ka.params_out[6 * s + q] = out.p[q];
      ka.chi2_out[s] = out.chi2;
      ka.iters_out[s] = out.iters;
      ka.status_out[s] = out.status;
      if (ka.evals_out) {
        ka.evals_out[2 * s] = out.n_grad;
        ka.evals_out[2 * s + 1] = out.n_trial;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launch table
// ---------------------------------------------------------------------------
// precision -> kernel: FP32 (float), MIXED (double), COMP (double, compensated sums)
template <int PPL>
static const void* kernel_ptr(int precision) {
  if (precision == SPOTFIT_PREC_MIXED)
    return reinterpret_cast<const void*>(&fit_wave_kernel<PPL, double, false>);
  if (precision == SPOTFIT_PREC_COMP)
    return reinterpret_cast<const void*>(&fit_wave_kernel<PPL, double, true>);
  return reinterpret_cast<const void*>(&fit_wave_kernel<PPL, float, false>);
}

template <int PPL>
static hipError_t launch_one(int precision, const KArgs& ka, int grid, hipStream_t st) {
  if (precision == SPOTFIT_PREC_MIXED)
    hipLaunchKernelGGL((fit_wave_kernel<PPL, double, false>), dim3(grid), dim3(64), 0, st, ka);
  else if (precision == SPOTFIT_PREC_COMP)
    hipLaunchKernelGGL((fit_wave_kernel<PPL, double, true>), dim3(grid), dim3(64), 0, st, ka);
  else
    hipLaunchKernelGGL((fit_wave_kernel<PPL, float, false>), dim3(grid), dim3(64), 0, st, ka);
  return hipGetLastError();
}

int ppl_for_pixels(int max_pixels) {
  int ppl = (max_pixels + 63) / 64;
  if (ppl <= 1) return 1;
  if (ppl <= 2) return 2;
  if (ppl <= 4) return 4;
  if (ppl <= 8) return 8;
  return 16;
}

const void* wave_kernel_symbol(int ppl, int precision) {
  switch (ppl) {
    case 1: return kernel_ptr<1>(precision);
    case 2: return kernel_ptr<2>(precision);
    case 4: return kernel_ptr<4>(precision);
    case 8: return kernel_ptr<8>(precision);
    default: return kernel_ptr<16>(precision);
  }
}

hipError_t launch_wave_kernel(int ppl, int precision, const KArgs& ka, int grid, hipStream_t st) {
  switch (ppl) {
    case 1: return launch_one<1>(precision, ka, grid, st);
    case 2: return launch_one<2>(precision, ka, grid, st);
    case 4: return launch_one<4>(precision, ka, grid, st);
    case 8: return launch_one<8>(precision, ka, grid, st);
    default: return launch_one<16>(precision, ka, grid, st);
  }
}

}  // namespace sf
