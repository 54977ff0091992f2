// spotfit_group.hip -- gfx950 kernel of the batched implicit-amplitude
// Levenberg-Marquardt Gaussian-spot fit (Leutenegger & Weber), separable form.
//
// Both profiles are separable: f(r, c) = ex(c) * ey(r) with
//   ex(c) = exp(-(c - x)^2 / (2 sx^2)),  ey(r) = exp(-(r - y)^2 / (2 sy^2))
// (Eq. 10 for sx = sy; axis-aligned elliptical otherwise).  Every sum the method
// needs (Eqs. 5-9) is therefore either a product of one-dimensional moments
// over columns and rows, or a bilinear form  sum_rc g(r,c) u(r) v(c)  that
// costs a few FMAs per pixel.  One evaluation takes W + H exponentials instead
// of W*H, and the whole evaluation is carried in double precision, so the
// chi^2 that decides every accept / retry / stop comparison is exact to
// ~1e-15 relative.
//
// Mapping: a group of L lanes (L = 8, 16 or 32) fits one spot with w, h <= L;
// 64/L spots share a wavefront.  In-group lane l owns column l (its h pixel
// values live in registers for the whole fit) and row l (it computes ey(l)).
// Per-group sums use the cross-lane tree of xlane.h (DPP / permlane).  The
// group's uniform state (parameters, sums, normal equations) lives in LDS, and
// the per-spot scalar work is spread over the group's lanes: lane j computes
// the derivative sums and amplitude derivatives of parameter j, lane t one
// entry of the normal matrix, before all lanes solve the 4x4 system.
//
// Per-group Levenberg-Marquardt state machine (Fit2DGaussian pseudo-code):
// every step of the wave loop evaluates each active group's candidate point
// (trial evaluation), takes that group's decisions, and then, only for groups
// that accepted a point, runs the derivative pass and the damped solve for the
// next candidate.  A group whose spot has stopped writes its results and
// fetches its next spot immediately, so groups never wait for each other's
// iteration counts.
//
// All spots are handled as (x, y, sx, sy).  For a symmetric spot sy == sx; its
// 3x3 system is the 4x4 elliptical one contracted along d/dsigma = d/dsx +
// d/dsy, padded with an identity row so every group solves a 4x4 system.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "xlane.h"

namespace sf {
namespace grp {

enum Mode : int { kNew = 0, kTrialFirst = 1, kTrialRetry = 2 };

__device__ __forceinline__ void lds_sync() {
  // orders this wavefront's LDS writes before its later LDS reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Uniform state of one group, in LDS.
template <int HM>
struct State {
  double pc[4];     // candidate point being evaluated
  double p[4];      // accepted point
  double best[4];   // point at the start of the iteration
  double delta[4];  // last step
  double A[10];     // normal matrix at best (upper triangle 00 01 02 03 11 12 13 22 23 33)
  double bv[4];     // right-hand side J^T (g - h) at best
  // evaluation at pc: one-dimensional sums, Eq. 5 sums, Eq. 6 amplitudes, Eq. 2 error
  double Sx, Sxx, Sy, Syy, F, FF, FG, D, a, b, chi;
  double chi_best, a_best, b_best;  // error and amplitudes at best
  double Gs, Tme;                   // sum g, MaxError threshold
  double ey[HM];                    // row factors at pc
  double red[16];                   // reduction results / moments
  double gd[4][5];                  // per parameter: dF, sum f df, dFG, d alpha, d beta
  double A4[14];                    // 4x4 normal matrix (elliptical) and right-hand side
};

// Totals over the group of the first K values; written to red[0..K-1].
template <int L, int K>
__device__ __forceinline__ void group_sums_to(double (&v)[K], double* red, int li) {
  constexpr int m = GroupLog<L>::m;
  group_halve<L, K>(v);
  const int rv = bitrev_bits(li, m);
  if constexpr (K >= L) {
#pragma unroll
    for (int i = 0; i < K / L; ++i) red[L * i + rv] = v[i];
  } else {
    if ((rv & ~(K - 1)) == 0) red[rv] = v[0];
  }
  lds_sync();
}

// Total over the group; every lane of the group holds it after the full tree.
template <int L>
__device__ __forceinline__ double group_sum1(double v) {
  double a[1] = {v};
  halve_from<6 - GroupLog<L>::m, 1>(a);
  return a[0];
}

__device__ __forceinline__ double clampn(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double pow10i(int k) {
  double t = 1.0;
  const int m = k < 0 ? -k : k;
  for (int i = 0; i < m; ++i) t *= 10.0;
  return k < 0 ? 1.0 / t : t;
}

// Cholesky solve of (A + lam diag A) d = bv, 4x4 symmetric (upper triangle in
// A[10]: 00 01 02 03 11 12 13 22 23 33).  NaN on a non-positive pivot.
__device__ __forceinline__ void solve4(const double* A, const double* bv, double lam, double* d) {
  const double m00 = A[0] + lam * A[0], m11 = A[4] + lam * A[4];
  const double m22 = A[7] + lam * A[7], m33 = A[9] + lam * A[9];
  bool ok = m00 > 0.0;
  const double l00 = sqrt(m00), i00 = 1.0 / l00;
  const double l10 = A[1] * i00, l20 = A[2] * i00, l30 = A[3] * i00;
  const double s11 = m11 - l10 * l10;
  ok = ok && s11 > 0.0;
  const double l11 = sqrt(s11), i11 = 1.0 / l11;
  const double l21 = (A[5] - l20 * l10) * i11, l31 = (A[6] - l30 * l10) * i11;
  const double s22 = m22 - l20 * l20 - l21 * l21;
  ok = ok && s22 > 0.0;
  const double l22 = sqrt(s22), i22 = 1.0 / l22;
  const double l32 = (A[8] - l30 * l20 - l31 * l21) * i22;
  const double s33 = m33 - l30 * l30 - l31 * l31 - l32 * l32;
  ok = ok && s33 > 0.0;
  const double l33 = sqrt(s33), i33 = 1.0 / l33;
  const double y0 = bv[0] * i00;
  const double y1 = (bv[1] - l10 * y0) * i11;
  const double y2 = (bv[2] - l20 * y0 - l21 * y1) * i22;
  const double y3 = (bv[3] - l30 * y0 - l31 * y1 - l32 * y2) * i33;
  const double d3 = y3 * i33;
  const double d2 = (y2 - l32 * d3) * i22;
  const double d1 = (y1 - l21 * d2 - l31 * d3) * i11;
  const double d0 = (y0 - l10 * d1 - l20 * d2 - l30 * d3) * i00;
  ok = ok && __builtin_isfinite(d0) && __builtin_isfinite(d1) && __builtin_isfinite(d2) &&
       __builtin_isfinite(d3);
  const double nanv = __builtin_nan("");
  d[0] = ok ? d0 : nanv;
  d[1] = ok ? d1 : nanv;
  d[2] = ok ? d2 : nanv;
  d[3] = ok ? d3 : nanv;
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

// red[] after the derivative-pass reduction (16 group sums):
//   1, 2      X1 = sum dx ex,  X2 = sum dx^2 ex          (X0 = sum ex from the trial)
//   3..6      Xq1..Xq4 = sum dx^k ex^2                    (Xq0 = sum ex^2)
//   7, 8      Y1 = sum dy ey,  Y2 = sum dy^2 ey           (Y0 = sum ey)
//   9..12     Yq1..Yq4 = sum dy^k ey^2                    (Yq0 = sum ey^2)
//   13, 14    B_x = sum dx ex t,  B_sx = sum dx^2 ex t    (t = sum_r g ey per column)
//   15, 0     B_y = sum ex t_y,   B_sy = sum ex t_yy      (t_y, t_yy: (r-y), (r-y)^2 weights)
template <int L, int WPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_group_kernel(KArgs ka) {
  constexpr int G = 64 / L;  // groups (spots in flight) per wavefront
  constexpr int HM = L;      // rows held per lane
  constexpr double kC0 = 0.5 * (HM - 1);  // row origin of the bilinear row moments
  constexpr int kChunk = 4;               // rows processed between scheduling barriers
  __shared__ State<HM> sts[G];

  const int lane = __lane_id();
  const int gi = lane / L;
  const int li = lane % L;
  State<HM>& S = sts[gi];
  const int64_t stride = (int64_t)gridDim.x * G;
  const KOpts o = ka.opt;
  const double tau = o.tie_tau;

  // ---- per-group control state (identical on the L lanes of a group) ----
  int64_t s = (int64_t)blockIdx.x * G + gi;
  int w = 0, h = 0, k = 0, it = 0, status = 0, mode = kNew, n_grad = 0, n_trial = 0;
  bool sym = true;
  // ---- per-lane data ----
  float g[HM];  // column li of the spot (0 outside the spot)
  double ex = 0.0, eyo = 0.0, tcol = 0.0, t1c = 0.0, t2c = 0.0;

  // Fetch the next spot of this group, writing BAD_INPUT for unusable ones.
  auto fetch = [&]() {
    while (s < ka.n) {
      const spotfit_shape_t sh = ka.sizes[s];
      const float* in = ka.init + 4 * s;
      const float i0 = in[0], i1 = in[1], i2 = in[2], i3 = in[3];
      const int mdl = sh.model;
      const bool ell = mdl == SPOTFIT_ELL;
      const bool bad = sh.w < 3 || sh.h < 3 || sh.w > L || sh.h > L ||
                       sh.w * sh.h > o.max_pixels || sh.w > o.max_side || sh.h > o.max_side ||
                       (mdl != SPOTFIT_SYM && !ell) || !__builtin_isfinite(i0) ||
                       !__builtin_isfinite(i1) || !__builtin_isfinite(i2) || !(i2 > 0.f) ||
                       (ell && (!__builtin_isfinite(i3) || !(i3 > 0.f)));
      if (!bad) {
        w = sh.w;
        h = sh.h;
        sym = !ell;
        S.pc[0] = i0;
        S.pc[1] = i1;
        S.pc[2] = i2;
        S.pc[3] = ell ? (double)i3 : (double)i2;
        const int64_t off = ka.offsets[s];
        double cs = 0.0;
#pragma unroll
        for (int r0 = 0; r0 < HM; r0 += kChunk) {
#pragma unroll
          for (int r = r0; r < r0 + kChunk; ++r) {
            float gv = 0.f;
            if (r < h && li < w) {
              gv = ka.dtype == SPOTFIT_U16
                       ? float(static_cast<const uint16_t*>(ka.data)[off + r * w + li])
                       : static_cast<const float*>(ka.data)[off + r * w + li];
            }
            g[r] = gv;
            cs += double(gv);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        S.Gs = group_sum1<L>(cs);
        S.Tme = o.max_error_per_px * double(w * h);
        k = o.lambda0_exp10;
        it = 0;
        status = SPOTFIT_MAX_ITER;
        mode = kNew;
        n_grad = n_trial = 0;
        return;
      }
      if (li == 0) {
        const float nanf = __builtin_nanf("");
#pragma unroll
        for (int q = 0; q < 6; ++q) ka.params_out[6 * s + q] = nanf;
        ka.chi2_out[s] = nanf;
        ka.iters_out[s] = 0;
        ka.status_out[s] = SPOTFIT_BAD_INPUT;
        if (ka.evals_out) {
          ka.evals_out[2 * s] = 0;
          ka.evals_out[2 * s + 1] = 0;
        }
      }
      s += stride;
    }
  };

  fetch();

  while (__builtin_amdgcn_ballot_w64(s < ka.n) != 0) {
    if (s < ka.n) {
      // ================= trial evaluation at pc (Eqs. 2, 5, 6, 10) =================
      {
        const double x = S.pc[0], y = S.pc[1], sx = S.pc[2], sy = S.pc[3];
        const double dxc = double(li) - x;
        const double dyr = double(li) - y;
        ex = li < w ? exp(-0.5 * (dxc * dxc) / (sx * sx)) : 0.0;
        eyo = li < h ? exp(-0.5 * (dyr * dyr) / (sy * sy)) : 0.0;
        S.ey[li] = eyo;
        lds_sync();
        // column sums of g ey, and the row moments needed by the derivative pass
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
        for (int r0 = 0; r0 < HM; r0 += kChunk) {
#pragma unroll
          for (int r = r0; r < r0 + kChunk; ++r) {
            const double u = double(g[r]) * S.ey[r];
            t0 += u;
            t1 = __builtin_fma(u, double(r) - kC0, t1);
            t2 = __builtin_fma(u, (double(r) - kC0) * (double(r) - kC0), t2);
          }
          __builtin_amdgcn_sched_barrier(0);  // bounds the rows in flight (registers)
        }
        tcol = t0;
        t1c = t1;
        t2c = t2;
        double v[8] = {ex, ex * ex, eyo, eyo * eyo, ex * t0, 0.0, 0.0, 0.0};
        group_sums_to<L, 8>(v, S.red, li);
        const double Sx = S.red[0], Sxx = S.red[1], Sy = S.red[2], Syy = S.red[3];
        const double FG = S.red[4];
        const double F = Sx * Sy, FF = Sxx * Syy;
        const double Nn = double(w * h), Gs = S.Gs;
        const double D = Nn * FF - F * F;
        const bool okD = D > 0.0 && __builtin_isfinite(D);
        const double iD = 1.0 / D;
        const double a = (Nn * FG - F * Gs) * iD;
        const double b = (Gs * FF - F * FG) * iD;
        // residual sum of squares, r = alpha f + beta - g over the spot's pixels
        // (the fence makes this loop re-read the row factors instead of keeping
        // all of them live in registers across the reduction)
        lds_sync();
        double c2 = 0.0;
        const double bm = li < w ? b : 0.0;
#pragma unroll
        for (int r0 = 0; r0 < HM; r0 += kChunk) {
#pragma unroll
          for (int r = r0; r < r0 + kChunk; ++r) {
            if (r < h) {
              const double res = __builtin_fma(a, ex * S.ey[r], bm - double(g[r]));
              c2 = __builtin_fma(res, res, c2);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        double chi = group_sum1<L>(c2);
        if (!okD || !__builtin_isfinite(chi) || !__builtin_isfinite(a) || !__builtin_isfinite(b))
          chi = __builtin_nan("");
        S.Sx = Sx;
        S.Sxx = Sxx;
        S.Sy = Sy;
        S.Syy = Syy;
        S.F = F;
        S.FF = FF;
        S.FG = FG;
        S.D = D;
        S.a = a;
        S.b = b;
        S.chi = chi;
      }
      if (mode != kNew) ++n_trial;

      // ================= decisions (Fit2DGaussian loop) =================
      bool start = false, do_grad = false, do_solve = false, done = false;
      if (mode == kNew) {
#pragma unroll
        for (int q = 0; q < 4; ++q) S.p[q] = S.pc[q];
        start = true;
      } else {
        const double Chi = S.chi, chi = S.chi_best;
        if (mode == kTrialFirst && Chi < chi * (1.0 - tau)) --k;  // improved: less damping
        bool small = true;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          small = small && ((sym && q == 3) || fabs(S.delta[q]) < o.min_step_rel * fabs(S.best[q]));
        const bool worse = chi * (1.0 + tau) < Chi;
        if (!small && worse && k < o.lambda_max_exp10) {
          ++k;  // more damping, retry from best
          mode = kTrialRetry;
          do_solve = true;
        } else if (worse || __builtin_isnan(Chi)) {
#pragma unroll
          for (int q = 0; q < 4; ++q) S.p[q] = S.best[q];
          S.a = S.a_best;
          S.b = S.b_best;
          S.chi = chi;
          status = SPOTFIT_NOT_CONVERGED;
          done = true;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) S.p[q] = S.pc[q];
          if (Chi < S.Tme) {
            status = SPOTFIT_MAX_ERROR;
            done = true;
          } else if (chi * (1.0 - o.min_delta) < Chi) {
            status = SPOTFIT_MIN_DELTA;
            done = true;
          } else if (small) {
            status = SPOTFIT_MIN_STEP;
            done = true;
          } else {
            start = true;
          }
        }
      }
      if (start) {  // a new iteration at the accepted point p (= pc)
        if (it >= o.max_iter) {
          status = SPOTFIT_MAX_ITER;
          done = true;
        } else {
          ++it;
          ++n_grad;
          const double chi = S.chi;
          if (__builtin_isnan(chi)) {
            status = SPOTFIT_NOT_CONVERGED;
            done = true;
          } else if (chi < S.Tme) {
            status = SPOTFIT_MAX_ERROR;
            done = true;
          } else {
            S.chi_best = chi;
            S.a_best = S.a;
            S.b_best = S.b;
#pragma unroll
            for (int q = 0; q < 4; ++q) S.best[q] = S.p[q];
            mode = kTrialFirst;
            do_grad = true;
            do_solve = true;
          }
        }
      }

      // ================= derivative pass at p (Eqs. 7-9, 11) =================
      if (do_grad) {
        const double x = S.p[0], y = S.p[1];
        // lane li: moments of column li and row li, bilinear terms of column li
        const double dx = double(li) - x, dy = double(li) - y;
        const double ex2 = ex * ex, ey2 = eyo * eyo;
        const double dx2 = dx * dx, dy2 = dy * dy;
        const double yc = y - kC0;
        const double t1y = t1c - yc * tcol;                        // sum_r (r-y) g ey
        const double t2y = t2c - 2.0 * yc * t1c + yc * yc * tcol;  // sum_r (r-y)^2 g ey
        double v[16] = {ex * t2y,        dx * ex,         dx2 * ex,        dx * ex2,
                        dx2 * ex2,       dx2 * dx * ex2,  dx2 * dx2 * ex2, dy * eyo,
                        dy2 * eyo,       dy * ey2,        dy2 * ey2,       dy2 * dy * ey2,
                        dy2 * dy2 * ey2, dx * ex * tcol,  dx2 * ex * tcol, ex * t1y};
        group_sums_to<L, 16>(v, S.red, li);
        const double isx = 1.0 / S.p[2], isy = 1.0 / S.p[3];
        const double Sx = S.Sx, Sy = S.Sy, Sxx = S.Sxx, Syy = S.Syy;
        const double Nn = double(w * h), Gs = S.Gs, iD = 1.0 / S.D;
        const double F = S.F, FF = S.FF, FG = S.FG, a = S.a, b = S.b;
        // --- lanes j < 4: sums of parameter j (Eq. 7) and Eq. 8 ---
        if (li < 4) {
          const int j = li;
          const int ox = ox_of(j), oy = oy_of(j);
          const double wj = j == 0 ? isx * isx : j == 1 ? isy * isy : j == 2 ? isx * isx * isx
                                                                             : isy * isy * isy;
          const double X = ox == 0 ? Sx : S.red[ox];
          const double Y = oy == 0 ? Sy : S.red[6 + oy];
          const double Xq = ox == 0 ? Sxx : S.red[2 + ox];
          const double Yq = oy == 0 ? Syy : S.red[8 + oy];
          const double Bj = S.red[j == 0 ? 13 : j == 1 ? 15 : j == 2 ? 14 : 0];
          const double dF = X * Y * wj;
          const double Sfd = Xq * Yq * wj;
          const double dFG = Bj * wj;
          const double dFF = 2.0 * Sfd;
          const double gam = Nn * dFF - 2.0 * F * dF;
          S.gd[j][0] = dF;
          S.gd[j][1] = Sfd;
          S.gd[j][2] = dFG;
          S.gd[j][3] = (Nn * dFG - Gs * dF - a * gam) * iD;
          S.gd[j][4] = (Gs * dFF - FG * dF - F * dFG - b * gam) * iD;
        }
        lds_sync();
        // --- lane t < 10: normal-matrix entry t; lanes 10..13: right-hand side ---
        // J_j = da_j f + a df_j + db_j  (Eq. 9, second factor)
        for (int t = li; t < 14; t += L) {
          double val;
          if (t < 10) {
            const int i = tri_i(t), j = tri_j(t);
            const double dai = S.gd[i][3], dbi = S.gd[i][4], daj = S.gd[j][3], dbj = S.gd[j][4];
            const int oxs = ox_of(i) + ox_of(j), oys = oy_of(i) + oy_of(j);
            const double Xq = oxs == 0 ? Sxx : S.red[2 + oxs];
            const double Yq = oys == 0 ? Syy : S.red[8 + oys];
            const double wi = i == 0 ? isx * isx : i == 1 ? isy * isy : i == 2 ? isx * isx * isx
                                                                               : isy * isy * isy;
            const double wj = j == 0 ? isx * isx : j == 1 ? isy * isy : j == 2 ? isx * isx * isx
                                                                               : isy * isy * isy;
            const double Sdd = Xq * Yq * wi * wj;  // sum df_i df_j
            val = dai * daj * FF + a * (dai * S.gd[j][1] + daj * S.gd[i][1]) +
                  (dai * dbj + dbi * daj) * F + a * a * Sdd +
                  a * (dbj * S.gd[i][0] + dbi * S.gd[j][0]) + Nn * dbi * dbj;
          } else {
            const int j = t - 10;
            const double sfr = a * FF + b * F - FG;  // sum f r  (0 up to rounding, Eq. 4)
            const double sr = a * F + b * Nn - Gs;   // sum r
            val = -(S.gd[j][3] * sfr + a * (a * S.gd[j][1] + b * S.gd[j][0] - S.gd[j][2]) +
                    S.gd[j][4] * sr);
          }
          S.A4[t] = val;
        }
        lds_sync();
        // --- symmetric spots: sigma = sx = sy, contract and pad with identity ---
        for (int t = li; t < 14; t += L) {
          double val = S.A4[t];
          if (sym) {
            if (t == 2 || t == 5 || t == 12) val += S.A4[t + 1];
            if (t == 7) val += 2.0 * S.A4[8] + S.A4[9];
            if (t == 3 || t == 6 || t == 8 || t == 13) val = 0.0;
            if (t == 9) val = 1.0;
          }
          if (t < 10)
            S.A[t] = val;
          else
            S.bv[t - 10] = val;
        }
        lds_sync();
      }

      // ================= damped step (Eq. 14) and limit() =================
      if (do_solve) {
        double d[4];
        solve4(S.A, S.bv, pow10i(k), d);
        const double smax = o.sigma_max_frac * double(w > h ? w : h);
        const double p2 = clampn(S.best[2] + d[2], o.sigma_min, smax);
        S.pc[0] = clampn(S.best[0] + d[0], -0.5, double(w) - 0.5);
        S.pc[1] = clampn(S.best[1] + d[1], -0.5, double(h) - 0.5);
        S.pc[2] = p2;
        S.pc[3] = sym ? p2 : clampn(S.best[3] + d[3], o.sigma_min, smax);
#pragma unroll
        for (int q = 0; q < 4; ++q) S.delta[q] = d[q];
      }

      // ================= results and the next spot =================
      if (done) {
        if (li == 0) {
          float* po = ka.params_out + 6 * s;
          po[0] = float(S.p[0]);
          po[1] = float(S.p[1]);
          po[2] = float(S.p[2]);
          po[3] = float(S.p[3]);
          po[4] = float(S.a);
          po[5] = float(S.b);
          ka.chi2_out[s] = float(S.chi);
          ka.iters_out[s] = it;
          ka.status_out[s] = status;
          if (ka.evals_out) {
            ka.evals_out[2 * s] = n_grad;
            ka.evals_out[2 * s + 1] = n_trial;
          }
        }
        s += stride;
        fetch();
      }
    }
  }
}

template <int L, int WPE>
static hipError_t launch_lw(const KArgs& ka, int grid, hipStream_t st) {
  hipLaunchKernelGGL((fit_group_kernel<L, WPE>), dim3(grid), dim3(64), 0, st, ka);
  return hipGetLastError();
}

template <int L>
static hipError_t launch_l(int wpe, const KArgs& ka, int grid, hipStream_t st) {
  switch (wpe) {
    case 2: return launch_lw<L, 2>(ka, grid, st);
    case 3: return launch_lw<L, 3>(ka, grid, st);
    case 4: return launch_lw<L, 4>(ka, grid, st);
    default: return launch_lw<L, 1>(ka, grid, st);
  }
}

template <int L>
static const void* symbol_l(int wpe) {
  switch (wpe) {
    case 2: return reinterpret_cast<const void*>(&fit_group_kernel<L, 2>);
    case 3: return reinterpret_cast<const void*>(&fit_group_kernel<L, 3>);
    case 4: return reinterpret_cast<const void*>(&fit_group_kernel<L, 4>);
    default: return reinterpret_cast<const void*>(&fit_group_kernel<L, 1>);
  }
}

}  // namespace grp

int group_lanes_for_side(int max_side) {
  if (max_side <= 8) return 8;
  if (max_side <= 16) return 16;
  return 32;
}

const void* group_kernel_symbol(int lanes, int wpe) {
  switch (lanes) {
    case 8: return grp::symbol_l<8>(wpe);
    case 16: return grp::symbol_l<16>(wpe);
    default: return grp::symbol_l<32>(wpe);
  }
}

hipError_t launch_group_kernel(int lanes, int wpe, const KArgs& ka, int grid, hipStream_t st) {
  switch (lanes) {
    case 8: return grp::launch_l<8>(wpe, ka, grid, st);
    case 16: return grp::launch_l<16>(wpe, ka, grid, st);
    default: return grp::launch_l<32>(wpe, ka, grid, st);
  }
}

}  // namespace sf
