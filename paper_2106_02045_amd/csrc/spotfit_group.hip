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
#include "spotfit_lm.h"
#include "spotfit_start.h"
#include "xlane.h"

namespace sf {
namespace grp {

using namespace lm;

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
  int64_t next;                     // next spot index, broadcast from the group's first lane
};

// Start values of one spot (ini::moment_init_spot), out of line: its registers
// are then not allocated across the fit's loop, which only saves what it keeps
// live around this call.
template <int L, int CPL>
__device__ __noinline__ void start_values_of(const void* data, int dtype, spotfit_shape_t sh,
                                             int64_t off, int li, float* o4) {
  ini::moment_init_spot<L, CPL>(data, dtype, sh, off, li, o4);
}

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

// red[] after the derivative-pass reduction (16 group sums):
//   1, 2      X1 = sum dx ex,  X2 = sum dx^2 ex          (X0 = sum ex from the trial)
//   3..6      Xq1..Xq4 = sum dx^k ex^2                    (Xq0 = sum ex^2)
//   7, 8      Y1 = sum dy ey,  Y2 = sum dy^2 ey           (Y0 = sum ey)
//   9..12     Yq1..Yq4 = sum dy^k ey^2                    (Yq0 = sum ey^2)
//   13, 14    B_x = sum dx ex t,  B_sx = sum dx^2 ex t    (t = sum_r g ey per column)
//   15, 0     B_y = sum ex t_y,   B_sy = sum ex t_yy      (t_y, t_yy: (r-y), (r-y)^2 weights)
//
// Template parameters: L lanes per spot, CPL columns (and rows) per lane, so a
// group holds spots with w, h <= L*CPL; WPE = minimum waves per SIMD the
// register allocation must allow.  RAW: each group computes its spot's start
// values when it takes the spot (centroid and second moments, as the
// start-value kernel does) and writes them to ka.init_out.
template <int L, int CPL, bool RAW, class Src>
__device__ __forceinline__ void fit_groups(const KArgs& ka, Src& src, State<L * CPL>* sts) {
  constexpr int G = 64 / L;       // groups (spots in flight) per wavefront
  constexpr int HM = L * CPL;     // largest side of a spot
  constexpr double kC0 = 0.5 * (HM - 1);  // row origin of the bilinear row moments
  constexpr int kChunk = 4;               // rows processed between scheduling barriers
  static_assert(HM % kChunk == 0, "chunking");

  const int lane = __lane_id();
  const int gi = lane / L;
  const int li = lane % L;
  State<HM>& S = sts[gi];
  const KOpts o = ka.opt;

  // ---- per-group control state (identical on the L lanes of a group) ----
  int64_t s = src.first(gi, li, S.next);
  int w = 0, h = 0, k = 0, it = 0, status = 0, mode = kNew, n_grad = 0, n_trial = 0;
  bool sym = true;
  // ---- per-lane data: columns li + L*j and rows li + L*j, j < CPL ----
  float g[CPL][HM];  // the lane's columns of the spot (0 outside the spot)
  double ex[CPL], eyo[CPL], tcol[CPL], t1c[CPL], t2c[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) ex[j] = eyo[j] = tcol[j] = t1c[j] = t2c[j] = 0.0;

  // The current spot's pixels into g (0 outside the spot); returns the lane's
  // sum of them.
  auto load_spot = [&](int64_t off) {
    double cs = 0.0;
#pragma unroll
    for (int r0 = 0; r0 < HM; r0 += kChunk) {
#pragma unroll
      for (int r = r0; r < r0 + kChunk; ++r) {
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const int c = li + L * j;
          float gv = 0.f;
          if (r < h && c < w) {
            gv = ka.dtype == SPOTFIT_U16
                     ? float(static_cast<const uint16_t*>(ka.data)[off + r * w + c])
                     : static_cast<const float*>(ka.data)[off + r * w + c];
          }
          g[j][r] = gv;
          cs += double(gv);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    return cs;
  };

  // Fetch the next spot of this group, writing BAD_INPUT for unusable ones.
  auto fetch = [&]() {
    while (s >= 0) {
      const spotfit_shape_t sh = ka.sizes[s];
      const int mdl = sh.model;
      const bool ell = mdl == SPOTFIT_ELL;
      const bool bad_shape = sh.w < 3 || sh.h < 3 || sh.w > HM || sh.h > HM ||
                             sh.w * sh.h > o.max_pixels || sh.w > o.max_side ||
                             sh.h > o.max_side || (mdl != SPOTFIT_SYM && !ell);
      const int64_t off = ka.offsets[s];
      const float nanf = __builtin_nanf("");
      float iv[4] = {nanf, nanf, nanf, nanf};
      if constexpr (RAW) {
        if (!bad_shape) start_values_of<L, CPL>(ka.data, ka.dtype, sh, off, li, iv);
        if (li == 0) {
          float* io = ka.init_out + 4 * s;
#pragma unroll
          for (int q = 0; q < 4; ++q) io[q] = iv[q];
        }
      } else {
        const float* in = ka.init + 4 * s;
#pragma unroll
        for (int q = 0; q < 4; ++q) iv[q] = in[q];
      }
      const bool bad = bad_shape || !__builtin_isfinite(iv[0]) || !__builtin_isfinite(iv[1]) ||
                       !__builtin_isfinite(iv[2]) || !(iv[2] > 0.f) ||
                       (ell && (!__builtin_isfinite(iv[3]) || !(iv[3] > 0.f)));
      if (!bad) {
        w = sh.w;
        h = sh.h;
        sym = !ell;
        S.pc[0] = iv[0];
        S.pc[1] = iv[1];
        S.pc[2] = iv[2];
        S.pc[3] = ell ? (double)iv[3] : (double)iv[2];
        const double cs = load_spot(off);
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
      s = src.next(s, li, S.next);
    }
  };

  fetch();

  while (__builtin_amdgcn_ballot_w64(s >= 0) != 0) {
    if (s >= 0) {
      // ================= trial evaluation at pc (Eqs. 2, 5, 6, 10) =================
      {
        const double x = S.pc[0], y = S.pc[1];
        const double hx = -0.5 * rcp_nr(S.pc[2] * S.pc[2]);
        const double hy = -0.5 * rcp_nr(S.pc[3] * S.pc[3]);
        double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        // the lane's 2 CPL factors at once (outside the spot too, then dropped):
        // their exponentials interleave instead of running one after another
        double arg[2 * CPL], fac[2 * CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const int c = li + L * j;
          const double dxc = double(c) - x, dyr = double(c) - y;
          arg[j] = dxc * dxc * hx;
          arg[CPL + j] = dyr * dyr * hy;
        }
        exp_neg_n<2 * CPL>(arg, fac);
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const int c = li + L * j;
          ex[j] = c < w ? fac[j] : 0.0;
          eyo[j] = c < h ? fac[CPL + j] : 0.0;
          S.ey[c] = eyo[j];
          v[0] += ex[j];
          v[1] = __builtin_fma(ex[j], ex[j], v[1]);
          v[2] += eyo[j];
          v[3] = __builtin_fma(eyo[j], eyo[j], v[3]);
        }
        lds_sync();
        // column sums of g ey, and the row moments needed by the derivative pass
        double t0[CPL], t1[CPL], t2[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) t0[j] = t1[j] = t2[j] = 0.0;
#pragma unroll
        for (int r0 = 0; r0 < HM; r0 += kChunk) {
#pragma unroll
          for (int r = r0; r < r0 + kChunk; ++r) {
            const double e = S.ey[r];
            constexpr double dummy = 0.0;
            (void)dummy;
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
              const double u = double(g[j][r]) * e;
              t0[j] += u;
              t1[j] = __builtin_fma(u, double(r) - kC0, t1[j]);
              t2[j] = __builtin_fma(u, (double(r) - kC0) * (double(r) - kC0), t2[j]);
            }
          }
          __builtin_amdgcn_sched_barrier(0);  // bounds the rows in flight (registers)
        }
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          tcol[j] = t0[j];
          t1c[j] = t1[j];
          t2c[j] = t2[j];
          v[4] = __builtin_fma(ex[j], t0[j], v[4]);
        }
        group_sums_to<L, 8>(v, S.red, li);
        const double Sx = S.red[0], Sxx = S.red[1], Sy = S.red[2], Syy = S.red[3];
        const double FG = S.red[4];
        const double F = Sx * Sy, FF = Sxx * Syy;
        const double Nn = double(w * h), Gs = S.Gs;
        const double D = Nn * FF - F * F;
        const bool okD = D > 0.0 && __builtin_isfinite(D);
        const double iD = rcp_nr(D);
        const double a = (Nn * FG - F * Gs) * iD;
        const double b = (Gs * FF - F * FG) * iD;
        // residual sum of squares, r = alpha f + beta - g over the spot's pixels
        // (the fence makes this loop re-read the row factors instead of keeping
        // all of them live in registers across the reduction)
        lds_sync();
        double aex[CPL], bm[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          aex[j] = a * ex[j];
          bm[j] = li + L * j < w ? b : 0.0;
        }
        double c2 = 0.0;
#pragma unroll
        for (int r0 = 0; r0 < HM; r0 += kChunk) {
#pragma unroll
          for (int r = r0; r < r0 + kChunk; ++r) {
            if (r < h) {
              const double e = S.ey[r];
#pragma unroll
              for (int j = 0; j < CPL; ++j) {
                const double res = __builtin_fma(aex[j], e, bm[j] - double(g[j][r]));
                c2 = __builtin_fma(res, res, c2);
              }
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
        if (mode == kTrialFirst && Chi < chi * o.one_minus_tau) --k;  // improved: less damping
        // MinStep: every step below min_step_rel of its parameter, the centre
        // measured from the centre of the ROI
        bool small = true;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double org = q == 0 ? 0.5 * double(w - 1) : q == 1 ? 0.5 * double(h - 1) : 0.0;
          small = small &&
                  ((sym && q == 3) || fabs(S.delta[q]) < o.min_step_rel * fabs(S.best[q] - org));
        }
        const bool worse = chi * o.one_plus_tau < Chi;
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
          } else if (chi * o.one_minus_min_delta < Chi) {
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
        const double yc = y - kC0;
        // lane li: moments of its columns and rows, bilinear terms of its columns
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const int c = li + L * j;
          const double dx = double(c) - x, dy = double(c) - y;
          const double ex2 = ex[j] * ex[j], ey2 = eyo[j] * eyo[j];
          const double dx2 = dx * dx, dy2 = dy * dy;
          const double t1y = t1c[j] - yc * tcol[j];                          // sum_r (r-y) g ey
          const double t2y = t2c[j] - 2.0 * yc * t1c[j] + yc * yc * tcol[j];  // sum_r (r-y)^2 g ey
          v[0] = __builtin_fma(ex[j], t2y, v[0]);
          v[1] = __builtin_fma(dx, ex[j], v[1]);
          v[2] = __builtin_fma(dx2, ex[j], v[2]);
          v[3] = __builtin_fma(dx, ex2, v[3]);
          v[4] = __builtin_fma(dx2, ex2, v[4]);
          v[5] = __builtin_fma(dx2 * dx, ex2, v[5]);
          v[6] = __builtin_fma(dx2 * dx2, ex2, v[6]);
          v[7] = __builtin_fma(dy, eyo[j], v[7]);
          v[8] = __builtin_fma(dy2, eyo[j], v[8]);
          v[9] = __builtin_fma(dy, ey2, v[9]);
          v[10] = __builtin_fma(dy2, ey2, v[10]);
          v[11] = __builtin_fma(dy2 * dy, ey2, v[11]);
          v[12] = __builtin_fma(dy2 * dy2, ey2, v[12]);
          v[13] = __builtin_fma(dx * ex[j], tcol[j], v[13]);
          v[14] = __builtin_fma(dx2 * ex[j], tcol[j], v[14]);
          v[15] = __builtin_fma(ex[j], t1y, v[15]);
        }
        group_sums_to<L, 16>(v, S.red, li);
        const double isx = rcp_nr(S.p[2]), isy = rcp_nr(S.p[3]);
        const double Sx = S.Sx, Sy = S.Sy, Sxx = S.Sxx, Syy = S.Syy;
        const double Nn = double(w * h), Gs = S.Gs, iD = rcp_nr(S.D);
        const double F = S.F, FF = S.FF, FG = S.FG, a = S.a, b = S.b;
        const double w0 = isx * isx, w1 = isy * isy, w2 = w0 * isx, w3 = w1 * isy;
        // --- lanes j < 4: sums of parameter j (Eq. 7) and Eq. 8 ---
        if (li < 4) {
          const int j = li;
          const int ox = ox_of(j), oy = oy_of(j);
          const double wj = j == 0 ? w0 : j == 1 ? w1 : j == 2 ? w2 : w3;
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
            const double wi = i == 0 ? w0 : i == 1 ? w1 : i == 2 ? w2 : w3;
            const double wj = j == 0 ? w0 : j == 1 ? w1 : j == 2 ? w2 : w3;
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
        s = src.next(s, li, S.next);
        fetch();
      }
    }
  }
}

// Spots s = first, first + stride, ... of a uniform batch (static striding).
struct StridedSrc {
  int64_t n, base, stride;
  __device__ int64_t first(int gi, int, int64_t&) const {
    const int64_t s = base + gi;
    return s < n ? s : -1;
  }
  __device__ int64_t next(int64_t s, int, int64_t&) const {
    s += stride;
    return s < n ? s : -1;
  }
};

template <int L, int CPL, int WPE, bool RAW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_group_kernel(KArgs ka) {
  constexpr int G = 64 / L;
  __shared__ State<L * CPL> sts[G];
  StridedSrc src{ka.n, (int64_t)blockIdx.x * G, (int64_t)gridDim.x * G};
  fit_groups<L, CPL, RAW>(ka, src, sts);
}


// ---------------------------------------------------------------------------
// Batches of uneven spot sizes: one persistent launch.
//
// A classify pass buckets the spot indices by size class (largest side <= 8,
// <= 16, <= 32) into per-class lists; the fit kernel then lets every wavefront
// run the plan (lanes per spot, columns per lane) of one class, its groups
// taking spots from that class's list through an atomic counter.  A wavefront
// whose class runs dry moves on to the next class, so no class waits for
// another's tail.  Result order is by spot index, independent of scheduling.
// ---------------------------------------------------------------------------
struct QueueSrc {
  const int32_t* list;  // spot indices of the class
  int32_t* take;        // next position to take (atomic)
  int32_t count;        // spots in the class
  __device__ int64_t pull(int li, int64_t& slot) const {
    if (li == 0) {
      const int32_t v = atomicAdd(take, 1);
      slot = v < count ? (int64_t)list[v] : -1;
    }
    lds_sync();
    const int64_t r = slot;
    lds_sync();
    return r;
  }
  __device__ int64_t first(int, int li, int64_t& slot) const { return pull(li, slot); }
  __device__ int64_t next(int64_t, int li, int64_t& slot) const { return pull(li, slot); }
};

__device__ __forceinline__ int size_class(const spotfit_shape_t& sh) {
  const int m = sh.w > sh.h ? sh.w : sh.h;
  return m <= 8 ? 0 : m <= 16 ? 1 : 2;
}

__device__ __forceinline__ int side_bucket(const spotfit_shape_t& sh) {
  const int m = sh.w > sh.h ? sh.w : sh.h;
  return m < kSortBuckets - 1 ? m : kSortBuckets - 1;
}

__device__ __forceinline__ int bucket_class(int b) { return b <= 8 ? 0 : b <= 16 ? 1 : 2; }

// Where each side's spots start in their class's list (buckets in increasing
// side), and the class totals: one thread.
__device__ __forceinline__ void bucket_offsets(const int* cnt, int* cursor, int32_t* counters) {
  int tot[3] = {0, 0, 0};
  for (int b = 0; b < kSortBuckets; ++b) {
    const int c = bucket_class(b);
    cursor[b] = tot[c];
    tot[c] += cnt[b];
  }
  for (int c = 0; c < 3; ++c) counters[c] = tot[c];
}

// Adds one to cnt[b] for every active lane with one LDS atomic per distinct
// bucket of the wavefront (a ballot counts the lanes of a bucket); returns the
// value cnt[b] had plus the lane's rank among the active lanes of its bucket.
// Called by whole wavefronts.
__device__ __forceinline__ int wave_bucket_add(int* cnt, int b, bool active) {
  const int lane = __lane_id();
  int res = 0;
  uint64_t todo = __builtin_amdgcn_ballot_w64(active);
  while (todo) {
    const int leader = (int)__builtin_ctzll(todo);
    const int bl = __builtin_amdgcn_readlane(b, leader);
    const bool in = active && b == bl;
    const uint64_t m = __builtin_amdgcn_ballot_w64(in);
    int base = 0;
    if (lane == leader) base = atomicAdd(&cnt[bl], __builtin_popcountll(m));
    base = __builtin_amdgcn_readlane(base, leader);
    if (in)
      res = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    todo &= ~m;
  }
  return res;
}

__global__ void mixed_reset_kernel(MixedWs ws) {
  if (threadIdx.x < 8) ws.counters[threadIdx.x] = 0;
  if (threadIdx.x < kSortWords) ws.sort[threadIdx.x] = 0;
}

// Small batches (serving frames): the whole counting sort in one workgroup
// (counts, offsets and the scatter in LDS), one launch.
__global__ __launch_bounds__(1024) void mixed_small_classify_kernel(const spotfit_shape_t* sizes,
                                                                    int64_t n, MixedWs ws) {
  __shared__ int cnt[kSortBuckets], cursor[kSortBuckets];
  if (threadIdx.x < 8) ws.counters[threadIdx.x] = 0;
  if (threadIdx.x < kSortBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int lane = __lane_id();
  for (int64_t w0 = threadIdx.x & ~63; w0 < n; w0 += blockDim.x) {
    const int64_t s = w0 + lane;
    const bool act = s < n;
    wave_bucket_add(cnt, act ? side_bucket(sizes[s]) : 0, act);
  }
  __syncthreads();
  if (threadIdx.x == 0) bucket_offsets(cnt, cursor, ws.counters);
  __syncthreads();
  for (int64_t w0 = threadIdx.x & ~63; w0 < n; w0 += blockDim.x) {
    const int64_t s = w0 + lane;
    const bool act = s < n;
    const int b = act ? side_bucket(sizes[s]) : 0;
    const int pos = wave_bucket_add(cursor, b, act);
    if (act) ws.lists[(int64_t)bucket_class(b) * ws.cap + pos] = (int32_t)s;
  }
}

// Large batches, pass 1: spots per larger side (block histograms in LDS).
__global__ __launch_bounds__(256) void mixed_count_kernel(const spotfit_shape_t* sizes, int64_t n,
                                                         MixedWs ws) {
  __shared__ int cnt[kSortBuckets];
  if (threadIdx.x < kSortBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); w0 < n; w0 += stride) {
    const int64_t s = w0 + __lane_id();
    const bool act = s < n;
    wave_bucket_add(cnt, act ? side_bucket(sizes[s]) : 0, act);
  }
  __syncthreads();
  if (threadIdx.x < kSortBuckets && cnt[threadIdx.x])
    atomicAdd(&ws.sort[threadIdx.x], cnt[threadIdx.x]);
}

// Pass 2: list offsets of the sides and class totals.
__global__ void mixed_offsets_kernel(MixedWs ws) {
  if (threadIdx.x == 0) bucket_offsets(ws.sort, ws.sort + 64, ws.counters);
}

// Pass 3: each block counts its spots per side again, reserves a range of every
// side's part of the list and writes its spots there (same spots, same order).
__global__ __launch_bounds__(256) void mixed_scatter_kernel(const spotfit_shape_t* sizes, int64_t n,
                                                           MixedWs ws) {
  __shared__ int cnt[kSortBuckets], base[kSortBuckets];
  if (threadIdx.x < kSortBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  for (int64_t w0 = first; w0 < n; w0 += stride) {
    const int64_t s = w0 + __lane_id();
    const bool act = s < n;
    wave_bucket_add(cnt, act ? side_bucket(sizes[s]) : 0, act);
  }
  __syncthreads();
  if (threadIdx.x < kSortBuckets) {
    base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&ws.sort[64 + threadIdx.x], cnt[threadIdx.x]) : 0;
    cnt[threadIdx.x] = 0;
  }
  __syncthreads();
  for (int64_t w0 = first; w0 < n; w0 += stride) {
    const int64_t s = w0 + __lane_id();
    const bool act = s < n;
    const int b = act ? side_bucket(sizes[s]) : 0;
    const int rank = wave_bucket_add(cnt, b, act);
    if (act) ws.lists[(int64_t)bucket_class(b) * ws.cap + base[b] + rank] = (int32_t)s;
  }
}

template <int L0, int C0, int L1, int C1, int L2, int C2, int WPE, bool RAW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_mixed_kernel(
    KArgs ka, MixedWs ws) {
  __shared__ union {
    State<L0 * C0> a[64 / L0];
    State<L1 * C1> b[64 / L1];
    State<L2 * C2> c[64 / L2];
  } st;
  // counters[0..2]: spots per class (filled by the classify pass), [3..5]: taken
  const int start = blockIdx.x % 3;
  for (int q = 0; q < 3; ++q) {
    const int c = (start + q) % 3;
    QueueSrc src{ws.lists + (int64_t)c * ws.cap, ws.counters + 3 + c, ws.counters[c]};
    if (c == 0)
      fit_groups<L0, C0, RAW>(ka, src, st.a);
    else if (c == 1)
      fit_groups<L1, C1, RAW>(ka, src, st.b);
    else
      fit_groups<L2, C2, RAW>(ka, src, st.c);
  }
}

template <int L, int CPL, int WPE>
static hipError_t launch_lw(const KArgs& ka, int grid, hipStream_t st) {
  if (ka.init_out)
    hipLaunchKernelGGL((fit_group_kernel<L, CPL, WPE, true>), dim3(grid), dim3(64), 0, st, ka);
  else
    hipLaunchKernelGGL((fit_group_kernel<L, CPL, WPE, false>), dim3(grid), dim3(64), 0, st, ka);
  return hipGetLastError();
}

template <int L, int CPL, int WPE>
static const void* sym_lw() {
  return reinterpret_cast<const void*>(&fit_group_kernel<L, CPL, WPE, false>);
}

// The compiled plans: (lanes per spot, columns per lane, min waves per SIMD).
// Entries 5 and 6 are entries 2 and 4 at one or two waves per SIMD, where they
// spill no registers (for batches too small to fill the chip); they are plan
// numbers 9 and 10, after the narrow plans 5..8.
#define SF_GROUP_PLANS(X) \
  X(0, 8, 1, 2)           \
  X(1, 8, 2, 2)           \
  X(2, 16, 1, 3)          \
  X(3, 16, 2, 2)          \
  X(4, 32, 1, 3)          \
  X(5, 16, 1, 1)          \
  X(6, 32, 1, 1)

}  // namespace grp

int wide_plan_count() { return 5; }

// The lane-owned plans: lanes per group, columns per lane, spots per group.
constexpr int kOwnedPlans = 5;
static const int kOwned[kOwnedPlans][3] = {{4, 4, 4}, {4, 4, 2}, {4, 2, 4}, {16, 2, 4}, {16, 2, 8}};

int group_plan_count() { return wide_plan_count() + narrow_plan_count() + 2 + kOwnedPlans; }

// Plan numbers: 0..4 wide, then the narrow plans, then the one-wave builds,
// then the lane-owned plans in kOwned's order.
static int owned_base() { return wide_plan_count() + narrow_plan_count() + 2; }
int owned_plan_id(int lanes, int cpl, int own) {
  for (int i = 0; i < kOwnedPlans; ++i)
    if (kOwned[i][0] == lanes && kOwned[i][1] == cpl && kOwned[i][2] == own) return owned_base() + i;
  return -1;
}
// index into kOwned, or -1
static int owned_of(int plan) {
  const int i = plan - owned_base();
  return i >= 0 && i < kOwnedPlans ? i : -1;
}
// the narrow plan of the same lanes x columns (4x2: plan 5, 4x4: 6, 16x2: 8)
int plan_for_raw(int plan) {
  const int i = owned_of(plan);
  if (i < 0) return plan;
  return wide_plan_count() + (kOwned[i][0] == 16 ? 3 : kOwned[i][1] == 2 ? 0 : 1);
}
static bool narrow_plan(int plan) {
  return plan >= wide_plan_count() && plan < wide_plan_count() + narrow_plan_count();
}
static int wide_entry(int plan) { return plan < wide_plan_count() ? plan : plan - narrow_plan_count(); }

void group_plan_shape(int plan, int* lanes, int* cpl) {
  if (narrow_plan(plan)) return narrow_plan_shape(plan - wide_plan_count(), lanes, cpl);
  if (const int i = owned_of(plan); i >= 0) {  // 64 / lanes spots per wavefront
    *lanes = kOwned[i][0] / kOwned[i][2];
    *cpl = kOwned[i][1] * kOwned[i][2];
    return;
  }
  plan = wide_entry(plan);
#define SF_SHAPE(I, L, C, W) \
  if (plan == I) {           \
    *lanes = L;              \
    *cpl = C;                \
    return;                  \
  }
  SF_GROUP_PLANS(SF_SHAPE)
#undef SF_SHAPE
  *lanes = 0;
  *cpl = 0;
}

const void* group_kernel_symbol(int plan) {
  if (narrow_plan(plan)) return narrow_kernel_symbol(plan - wide_plan_count());
  if (const int i = owned_of(plan); i >= 0) return owned_kernel_symbol(kOwned[i][0], kOwned[i][1], kOwned[i][2]);
  plan = wide_entry(plan);
#define SF_SYM(I, L, C, W) \
  if (plan == I) return grp::sym_lw<L, C, W>();
  SF_GROUP_PLANS(SF_SYM)
#undef SF_SYM
  return nullptr;
}

hipError_t launch_group_kernel(int plan, const KArgs& ka, int grid, hipStream_t st) {
  if (narrow_plan(plan)) return launch_narrow_kernel(plan - wide_plan_count(), ka, grid, st);
  if (const int i = owned_of(plan); i >= 0) {
    if (ka.init_out) return hipErrorInvalidValue;  // start values in the launch: plan_for_raw
    return launch_owned_kernel(kOwned[i][0], kOwned[i][1], kOwned[i][2], ka, grid, st);
  }
  plan = wide_entry(plan);
#define SF_LAUNCH(I, L, C, W) \
  if (plan == I) return grp::launch_lw<L, C, W>(ka, grid, st);
  SF_GROUP_PLANS(SF_LAUNCH)
#undef SF_LAUNCH
  return hipErrorInvalidValue;
}

// Mixed-size plans: plans of the classes (<= 8, <= 16, <= 32 px side).  Plan 3
// is plan 0 at one wave per SIMD: no register spills, for batches too small to
// fill the chip (the latency hint's choice up to kLeanMaxSpots spots).
#define SF_MIXED_PLANS(X)       \
  X(0, 8, 1, 16, 1, 32, 1, 3)   \
  X(1, 8, 1, 8, 2, 32, 1, 2)    \
  X(2, 8, 1, 16, 1, 16, 2, 2)   \
  X(3, 8, 1, 16, 1, 32, 1, 1)

int wide_mixed_plan_count() { return 4; }

int mixed_plan_count() { return wide_mixed_plan_count() + narrow_mixed_plan_count(); }

// narrow mixed plans 2 and 3 (lane-owned classes) -> narrow mixed plan 0
int mixed_plan_narrow(int plan) {
  const int i = plan - wide_mixed_plan_count();
  return i == 2 || i == 3 ? wide_mixed_plan_count() : plan;
}

const void* mixed_kernel_symbol(int plan) {
  if (plan >= wide_mixed_plan_count()) return narrow_mixed_kernel_symbol(plan - wide_mixed_plan_count());
#define SF_MSYM(I, A, B, C, D, E, F, W) \
  if (plan == I) return reinterpret_cast<const void*>(&grp::fit_mixed_kernel<A, B, C, D, E, F, W, false>);
  SF_MIXED_PLANS(SF_MSYM)
#undef SF_MSYM
  return nullptr;
}

hipError_t launch_mixed(int plan, const KArgs& ka, const MixedWs& ws, int grid, hipStream_t st) {
  hipError_t e;
  if (!ws.sort) return hipErrorInvalidValue;
  if (ka.n <= 65536) {
    hipLaunchKernelGGL(grp::mixed_small_classify_kernel, dim3(1), dim3(1024), 0, st, ka.sizes, ka.n, ws);
    e = hipGetLastError();
  } else {
    // at most 1024 blocks, each going over its share of the spots a wavefront at a time
    const int64_t cb = (ka.n + 255) / 256 < 1024 ? (ka.n + 255) / 256 : 1024;
    hipLaunchKernelGGL(grp::mixed_reset_kernel, dim3(1), dim3(kSortWords), 0, st, ws);
    e = hipGetLastError();
    if (e == hipSuccess) {
      hipLaunchKernelGGL(grp::mixed_count_kernel, dim3((unsigned)cb), dim3(256), 0, st, ka.sizes,
                         ka.n, ws);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(grp::mixed_offsets_kernel, dim3(1), dim3(64), 0, st, ws);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(grp::mixed_scatter_kernel, dim3((unsigned)cb), dim3(256), 0, st, ka.sizes,
                         ka.n, ws);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return e;
  return launch_mixed_fit(plan, ka, ws, grid, st);
}

hipError_t launch_mixed_fit(int plan, const KArgs& ka, const MixedWs& ws, int grid, hipStream_t st) {
  if (plan >= wide_mixed_plan_count())
    return launch_narrow_mixed_fit(plan - wide_mixed_plan_count(), ka, ws, grid, st);
#define SF_MLAUNCH(I, A, B, C, D, E, F, W)                                                          \
  if (plan == I) {                                                                                  \
    if (ka.init_out)                                                                                \
      hipLaunchKernelGGL((grp::fit_mixed_kernel<A, B, C, D, E, F, W, true>), dim3(grid), dim3(64), \
                         0, st, ka, ws);                                                            \
    else                                                                                            \
      hipLaunchKernelGGL((grp::fit_mixed_kernel<A, B, C, D, E, F, W, false>), dim3(grid), dim3(64), \
                         0, st, ka, ws);                                                            \
    return hipGetLastError();                                                                       \
  }
  SF_MIXED_PLANS(SF_MLAUNCH)
#undef SF_MLAUNCH
  return hipErrorInvalidValue;
}

}  // namespace sf
