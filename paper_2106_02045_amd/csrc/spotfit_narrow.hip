// spotfit_narrow.hip -- gfx950 kernel of the batched implicit-amplitude
// Levenberg-Marquardt Gaussian-spot fit, separable form, narrow lane groups.
//
// The arithmetic is that of the separable kernel (f(r, c) = ex(c) * ey(r) for
// Eq. 10 and its axis-aligned elliptical form, every sum of Eqs. 5-9 as
// one-dimensional moments or bilinear forms, all in double precision).  What
// differs is the mapping: a spot is held by a small group of L = 4, 8 or 16
// lanes.
//
//  * Lane l of a group owns the columns c = l + L*j (j < CPL) with all their
//    rows: the CPL*HM raw pixel values stay in registers for the whole fit and
//    are converted where used.  It computes ex(c) for its columns and ey(r)
//    for the rows r = l + L*j; a pass over the pixels fetches each row's factor
//    from the lane that holds it by a DPP (or ds_swizzle) broadcast when it
//    reaches the row.
//  * The per-spot scalar state is identical on the L lanes: each lane takes
//    every scalar step itself, and the iteration state lives in LDS, each lane
//    reading back only its own writes, so no barriers are needed.
//  * Group totals are log2(L) DPP butterfly steps; the two partners add the
//    same two numbers, so every lane of a group holds bitwise the same total
//    and takes the same branch.
//
// One trial evaluation costs per lane 2*CPL exponentials and one pass over
// the pixels it owns: the column sums t(c) = sum_r g ey and the row sums
// s(r) = sum_c g ex, which give **G** and the derivative bilinear forms.  For
// 16-bit data chi^2 then follows from those sums and the exact per-spot
// N sum g^2 - G^2 (Eq. 2 at the amplitudes of Eq. 6); float data takes a
// second pass for the residual sum of squares.
//
// The Levenberg-Marquardt loop is the same flattened per-group state machine
// as the wide kernel (Fit2DGaussian pseudo-code): every wave step evaluates
// each active group's candidate, takes its decisions, then runs the
// derivative pass and the damped solve only where needed; a group whose spot
// stops writes its result and fetches its next spot at once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "lanegroup.h"
#include "spotfit_lm.h"
#include "spotfit_start.h"
#include "separable.h"
#include "spotfit_owned.h"

namespace sf {
namespace nrw {

using namespace lm;
using namespace lg;
using namespace sep;

// Zeros that the loads of a column outside a spot read instead (one row offset
// of a 32 x 32 spot at most, as float or as 16-bit values).  Never written.  Not
// const: a constant-memory array would make its pointer and the pixel pointer
// meet in the generic address space, turning every pixel load into a FLAT load
// (which also holds up every later LDS wait).
__device__ float kZeros[32 * 32];

// The spots a launch fits: queue position i (0 <= i < count) is spot list[i],
// or spot i itself when list is null.  Wavefronts reserve positions from the
// shared counter a chunk at a time and hand them to their groups one by one as
// the groups finish spots, so every group stays busy until the queue is empty
// (a fixed share per group leaves the fastest groups idle at the end).
struct SpotQueue {
  const int32_t* list;
  int32_t* take;
  int32_t count;
};

// Per-group state kept in LDS between the steps of an iteration.
struct NState {
  double A[10];   // normal matrix at best (upper triangle 00 01 02 03 11 12 13 22 23 33)
  double bv[4];   // right-hand side J^T (g - h) at best
  double best[4];  // point at the start of the iteration
  double chi_best, a_best, b_best;
  double chib_err;  // error bound of chi_best (0: summed directly)
  double cand[4];   // the candidate while the best point is re-evaluated
  int mode_saved;   // the mode whose decision a re-evaluation completes
  // sums of the evaluation at pc that the derivative pass reuses
  double Sx, Sxx, Sy, Syy, FG, D, Bx, Bsx, By, Bsy;
};

// Start values of one spot (ini::moment_init_spot), out of line: its registers
// are then not allocated across the fit's loop, which only saves what it keeps
// live around this call.
template <int L, int CPL, int DT>
__device__ __noinline__ void start_values_of(const void* data, spotfit_shape_t sh, int64_t off,
                                             int li, float* o4) {
  ini::moment_init_spot<L, CPL>(data, DT, sh, off, li, o4);
}

// Fit every spot the source hands to this wavefront's groups.
// L lanes per spot, CPL columns per lane: spots with w, h <= L * CPL; pixel
// data type DT (SPOTFIT_U16 or SPOTFIT_F32).  RAW: the start values are
// computed here (centroid and second moments, as the start-value kernel does)
// and written to ka.init_out; cinit is LDS for two chunks of them.
template <int L, int CPL, int DT, bool RAW>
__device__ __forceinline__ void fit_narrow(const KArgs& ka, const SpotQueue& q, NState* sts,
                                           float4* cinit) {
  constexpr int HM = L * CPL;
  const int lane = __lane_id();
  const int gi = lane / L;
  const int li = lane % L;
  const KOpts o = ka.opt;

  int64_t s = -1;  // the group's current spot
  int w = 0, h = 0, k = 0, it = 0, status = 0, mode = kNew, n_grad = 0, n_trial = 0;
  bool bad = false;  // the current spot is unusable: it ends at its first step as BAD_INPUT
  bool sym = true, small = false;

  // pixels of the lane's columns as loaded (0 outside the spot); converted where
  // used, so that no instruction of the fetch waits for the loads
  uint32_t g[CPL][HM];
  double ex[CPL], eyl[CPL];  // column factors of its columns, row factors of its rows
  double pc[4] = {0.0, 0.0, 0.0, 0.0};  // candidate point (accepted point after a decision)
  double a = 0.0, b = 0.0, chi = 0.0;   // Eq. 6 amplitudes and Eq. 2 error at pc
  double Gs = 0.0, Tme = 0.0;
  double Vs = 0.0;       // 16-bit data: N sum g^2 - G^2 of the spot (exact)
  double chi_err = 0.0;  // bound on |chi - chi summed over the pixels|
#pragma unroll
  for (int j = 0; j < CPL; ++j) ex[j] = eyl[j] = 0.0;
  // Iteration state and the sums of the last evaluation, in LDS.  Every lane of
  // a group computes the same values and writes them itself, so each lane only
  // ever reads back its own writes: no synchronisation is needed.
  NState& S = sts[gi];

  // Each group holds a reserved next spot whose description (shape, offset,
  // start values) is loaded one spot ahead, so that taking a spot never waits.
  int64_t ns = -1;
  spotfit_shape_t nsh{0, 0, 0, 0};
  int64_t noff = 0;
  float4 nin = make_float4(0.f, 0.f, 0.f, 0.f);

  // Queue positions: the wavefront's current chunk [cbase, cbase + kChunk) of
  // which cused are handed out, and the next chunk, requested from the counter
  // once half of the current one is out (its base, in lane 0, is normally back
  // before it is needed).  A chunk is one position per group, so that a small
  // batch spreads over many wavefronts instead of queueing on a few.
  constexpr int kChunk = 64 / L;
  int cbase = 0, cused = 0, nbase_l0 = 0;
  bool nb_asked = false;
  // RAW: the wavefront computes the start values of a whole chunk at once, every
  // group one spot with all lanes active, into cinit[kChunk * buffer + position
  // in the chunk]; buffer cb holds the current chunk's, the other the next
  // chunk's once its base is known (nb_ready).
  int cb = 0;
  bool nb_ready = false;
  auto chunk_start = [&](int base, int buf) {
    const int p = base + gi;
    const int64_t id =
        (uint32_t)p < (uint32_t)q.count ? (q.list ? (int64_t)q.list[p] : (int64_t)p) : -1;
    const float nanf = __builtin_nanf("");
    float o4[4] = {nanf, nanf, nanf, nanf};
    if (id >= 0) {
      const spotfit_shape_t sh = ka.sizes[id];
      if (ini::usable<HM>(sh, o.max_side, o.max_pixels))
        start_values_of<L, CPL, DT>(ka.data, sh, ka.offsets[id], li, o4);
      if (li == 0) {
        float* io = ka.init_out + 4 * id;
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) io[q2] = o4[q2];
      }
    }
    if (li == 0) cinit[kChunk * buf + gi] = make_float4(o4[0], o4[1], o4[2], o4[3]);
    wave_lds_sync();
  };
  {
    int b0 = 0;
    if (lane == 0) b0 = atomicAdd(q.take, kChunk);
    cbase = __builtin_amdgcn_readfirstlane(b0);
  }
  if constexpr (RAW) chunk_start(cbase, 0);
  // Give every group with `want` a new reserved spot.  Called with the whole
  // wavefront active (the chunk state is wavefront-uniform).
  auto reserve = [&](bool want) {
    const bool req = want && li == 0;
    const uint64_t m = __builtin_amdgcn_ballot_w64(req);
    const int nreq = __builtin_popcountll(m);
    if constexpr (RAW) {
      // the next chunk's start values as soon as its base is back (or now, when
      // this call already takes from it)
      if (!nb_asked && cused + nreq > kChunk) {
        if (lane == 0) nbase_l0 = atomicAdd(q.take, kChunk);
        nb_asked = true;
      }
      if (nb_asked && !nb_ready) {
        chunk_start(__builtin_amdgcn_readfirstlane(nbase_l0), cb ^ 1);
        nb_ready = true;
      }
    }
    if (nreq == 0) return;
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    int pos, slot = 0;
    if (cused + nreq > kChunk) {  // nreq <= kChunk: the rest comes from the next chunk
      if (!nb_asked && lane == 0) nbase_l0 = atomicAdd(q.take, kChunk);
      const int nb = __builtin_amdgcn_readfirstlane(nbase_l0);
      const bool here = cused + rank < kChunk;
      pos = here ? cbase + cused + rank : nb + (cused + rank - kChunk);
      if constexpr (RAW) {
        slot = here ? kChunk * cb + cused + rank : kChunk * (cb ^ 1) + (cused + rank - kChunk);
        cb ^= 1;
        nb_ready = false;
      }
      cbase = nb;
      cused = cused + nreq - kChunk;
      nb_asked = false;
    } else {
      pos = cbase + cused + rank;
      if constexpr (RAW) slot = kChunk * cb + cused + rank;
      cused += nreq;
    }
    if (!nb_asked && 2 * cused >= kChunk) {
      if (lane == 0) nbase_l0 = atomicAdd(q.take, kChunk);
      nb_asked = true;
    }
    const int p = gbcast_i<L, 0>(req ? pos : 0);
    const int sl = RAW ? gbcast_i<L, 0>(req ? slot : 0) : 0;
    if (want) {
      ns = (uint32_t)p < (uint32_t)q.count ? (q.list ? (int64_t)q.list[p] : (int64_t)p) : -1;
      if (ns >= 0) {
        nsh = ka.sizes[ns];
        noff = ka.offsets[ns];
        if constexpr (RAW) {
          nin = cinit[sl];
        } else {
          const float* in = ka.init + 4 * ns;
          nin = make_float4(in[0], in[1], in[2], in[3]);
        }
      }
    }
  };

  // Take the reserved spot (its description only); an unusable one is marked
  // and ends at its next step with BAD_INPUT.
  int64_t off = 0;  // element offset of the current spot's pixels
  auto advance = [&]() {
    s = ns;
    ns = -1;
    if (s < 0) return;
    const spotfit_shape_t sh = nsh;
    const float i0 = nin.x, i1 = nin.y, i2 = nin.z, i3 = nin.w;
    off = noff;
    const int mdl = sh.model;
    const bool ell = mdl == SPOTFIT_ELL;
    bad = sh.w < 3 || sh.h < 3 || sh.w > HM || sh.h > HM || sh.w * sh.h > o.max_pixels ||
          sh.w > o.max_side || sh.h > o.max_side || (mdl != SPOTFIT_SYM && !ell) ||
          !__builtin_isfinite(i0) || !__builtin_isfinite(i1) || !__builtin_isfinite(i2) ||
          !(i2 > 0.f) || (ell && (!__builtin_isfinite(i3) || !(i3 > 0.f)));
    w = bad ? 0 : sh.w;
    h = bad ? 0 : sh.h;
    sym = !ell;
    pc[0] = i0;
    pc[1] = i1;
    pc[2] = i2;
    pc[3] = ell ? (double)i3 : (double)i2;
    Tme = o.max_error_per_px * double(w * h);
    k = o.lambda0_exp10;
    it = 0;
    status = SPOTFIT_MAX_ITER;
    mode = kNew;
    n_grad = n_trial = 0;
  };

  // The current spot's pixels into g, every slot at once and with no predicated
  // load: a column outside the spot reads a block of zeros, a row below it
  // repeats the spot's last row (every pass skips rows >= h).  Every wave step
  // reloads them (a spot that stays is read again from the cache), so that g
  // is never merged with an older value: no instruction waits for these loads
  // before the next trial evaluation reads them.
  auto load_pixels = [&]() {
    const int hh = h > 0 ? h : 1;
    if constexpr (DT == SPOTFIT_U16) {
      const uint16_t* zero = reinterpret_cast<const uint16_t*>(kZeros);
      const uint16_t* cp[CPL];  // top of each of the lane's columns
#pragma unroll
      for (int j = 0; j < CPL; ++j)
        cp[j] = li + L * j < w ? static_cast<const uint16_t*>(ka.data) + off + li + L * j : zero;
      // row offsets in bytes by additions (no multiply per row): rows below the
      // spot stay on its last row
      const uint32_t step = 2u * uint32_t(w), last = uint32_t(hh - 1) * step;
      uint32_t rb = 0;
#pragma unroll
      for (int r = 0; r < HM; ++r) {
        if (r > 0) rb = __builtin_elementwise_min(rb + step, last);
#pragma unroll
        for (int j = 0; j < CPL; ++j)
          g[j][r] = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(cp[j]) + rb);
      }
    } else {
      const uint32_t* zero = reinterpret_cast<const uint32_t*>(kZeros);
      const uint32_t* cp[CPL];
#pragma unroll
      for (int j = 0; j < CPL; ++j)
        cp[j] = li + L * j < w ? static_cast<const uint32_t*>(ka.data) + off + li + L * j : zero;
      const uint32_t step = 4u * uint32_t(w), last = uint32_t(hh - 1) * step;
      uint32_t rb = 0;
#pragma unroll
      for (int r = 0; r < HM; ++r) {
        if (r > 0) rb = __builtin_elementwise_min(rb + step, last);
#pragma unroll
        for (int j = 0; j < CPL; ++j)
          g[j][r] = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(cp[j]) + rb);
      }
    }
  };

  reserve(true);
  advance();
  reserve(true);
  load_pixels();

  while (__builtin_amdgcn_ballot_w64(s >= 0) != 0) {
    bool took = false;
    if (s >= 0 && bad) {
      if (li == 0) {
        const float nanf = __builtin_nanf("");
#pragma unroll
        for (int q2 = 0; q2 < 6; ++q2) ka.params_out[6 * s + q2] = nanf;
        ka.chi2_out[s] = nanf;
        ka.iters_out[s] = 0;
        ka.status_out[s] = SPOTFIT_BAD_INPUT;
        if (ka.evals_out) {
          ka.evals_out[2 * s] = 0;
          ka.evals_out[2 * s + 1] = 0;
        }
      }
      advance();
      took = true;
      if (s >= 0) load_pixels();
    } else if (s >= 0) {
      // ================= trial evaluation at pc (Eqs. 2, 5, 6, 10) =================
      {
        const double x = pc[0], y = pc[1];
        const double hx = -0.5 * rcp_nr(pc[2] * pc[2]);
        const double hy = -0.5 * rcp_nr(pc[3] * pc[3]);
        double sxp = 0.0, sxxp = 0.0, syp = 0.0, syyp = 0.0;
        // all 2 CPL factors at once, outside the spot too (then dropped), so
        // that their exponentials interleave instead of running one by one
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
          eyl[j] = c < h ? fac[CPL + j] : 0.0;
          sxp += ex[j];
          sxxp = __builtin_fma(ex[j], ex[j], sxxp);
          syp += eyl[j];
          syyp = __builtin_fma(eyl[j], eyl[j], syyp);
        }
        // column sums t(c) = sum_r g ey and row sums s(r) = sum_c g ex (lane's columns);
        // **G** = sum_r ey s(r), and the row-weighted forms of the derivative pass;
        // each row factor is fetched from its lane when its row is reached
        double t[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) t[j] = 0.0;
        double gp = 0.0, byp = 0.0, bsyp = 0.0, gsum_px = 0.0, ggp = 0.0;
        uint32_t gsi = 0;
        for_rows<L, CPL, HM>(eyl, [&](int r, double e) {
          if (r < h) {
            double sr = 0.0;
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
              const double gd = pixel<DT>(g[j][r]);
              t[j] = __builtin_fma(gd, e, t[j]);
              sr = __builtin_fma(gd, ex[j], sr);
              if constexpr (DT == SPOTFIT_U16) {
                gsi += g[j][r];                 // sum g (integer)
                ggp = __builtin_fma(gd, gd, ggp);  // sum g^2 (exact: integers below 2^53)
              } else {
                gsum_px += gd;
              }
            }
            // moments about row 0 (r and r^2 are constants of the unrolled
            // loop); shifted to the spot's centre after the group totals
            const double es = e * sr;
            gp += es;
            byp = __builtin_fma(double(r), es, byp);
            bsyp = __builtin_fma(double(r * r), es, bsyp);
          }
        });
        double bxp = 0.0, bsxp = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const double dx = double(li + L * j) - x;
          const double et = ex[j] * t[j];
          bxp = __builtin_fma(dx, et, bxp);
          bsxp = __builtin_fma(dx * dx, et, bsxp);
        }
        const double Nn = double(w * h);
        if (mode == kNew) {  // per-spot constants of a new spot
          if constexpr (DT == SPOTFIT_U16) {
            Gs = double(gsum_i<L>((int)gsi));
            Vs = Nn * gsum<L>(ggp) - Gs * Gs;  // every step exact
          } else {
            Gs = gsum<L>(gsum_px);
          }
        }
        const double Sx = gsum<L>(sxp), Sxx = gsum<L>(sxxp);
        const double Sy = gsum<L>(syp), Syy = gsum<L>(syyp);
        const double FG = gsum<L>(gp);
        S.Bx = gsum<L>(bxp);
        S.Bsx = gsum<L>(bsxp);
        {
          const double R1 = gsum<L>(byp), R2 = gsum<L>(bsyp);  // sum r e s(r), sum r^2 e s(r)
          S.By = __builtin_fma(-y, FG, R1);                       // sum (r - y) e s(r)
          S.Bsy = __builtin_fma(-y, __builtin_fma(2.0, R1, -y * FG), R2);  // sum (r - y)^2 e s(r)
        }
        const Amplitudes am = amplitudes(Nn, Sx, Sxx, Sy, Syy, FG, Gs);
        const double D = am.D;
        S.Sx = Sx;
        S.Sxx = Sxx;
        S.Sy = Sy;
        S.Syy = Syy;
        S.FG = FG;
        S.D = D;
        const bool okD = D > 0.0 && __builtin_isfinite(D);
        a = am.a;
        b = am.b;
        // direct sum over the pixels: always for float data; for 16-bit data
        // only where a close decision is being re-taken
        bool direct = DT != SPOTFIT_U16;
        if constexpr (DT == SPOTFIT_U16) {
          chi_closed(Vs, am, Nn, FG, Gs, w, h, chi, chi_err);  // Eq. 2, no second pixel pass
          direct = mode == kRecheckBest || mode == kRecheckCand;
        }
        if (__builtin_amdgcn_ballot_w64(direct) != 0 && direct) {
          // the residual sum of squares, r = alpha f + beta - g
          double aex[CPL], bm[CPL], c2[CPL];
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            aex[j] = a * ex[j];
            bm[j] = li + L * j < w ? b : 0.0;
            c2[j] = 0.0;
          }
          for_rows<L, CPL, HM>(eyl, [&](int r, double e) {
            if (r < h) {
#pragma unroll
              for (int j = 0; j < CPL; ++j) {
                // a fresh conversion: reusing the first pass's doubles would keep
                // all CPL*HM of them live in registers
                uint32_t gv = g[j][r];
                asm("" : "+v"(gv));
                const double res = __builtin_fma(aex[j], e, bm[j] - pixel<DT>(gv));
                c2[j] = __builtin_fma(res, res, c2[j]);
              }
            }
          });
          double c2s = c2[0];
#pragma unroll
          for (int j = 1; j < CPL; ++j) c2s += c2[j];
          chi = gsum<L>(c2s);
          chi_err = 0.0;
        }
        if (!okD || !__builtin_isfinite(chi) || !__builtin_isfinite(a) || !__builtin_isfinite(b))
          chi = __builtin_nan("");
      }
      if (mode == kTrialFirst || mode == kTrialRetry) ++n_trial;

      // ================= decisions (Fit2DGaussian loop) =================
      bool start = false, do_grad = false, do_solve = false, done = false, out_best = false;
      bool decide = true;
      if (mode == kRecheckBest) {
        // the best point's chi^2, summed directly; then the candidate's
        S.chi_best = chi;
        S.chib_err = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) pc[q] = S.cand[q];
        mode = kRecheckCand;
        decide = false;
      } else if (mode == kRecheckCand) {
        mode = S.mode_saved;  // chi is now summed directly: take the decision
      } else if (chi_err > 0.0) {
        // a decision closer to its threshold than the closed form's error
        // bound is re-taken with chi^2 summed directly (the best point's too
        // when that comparison involves it), so that every decision is the
        // one a direct sum takes
        const double chib = S.chi_best, eb = S.chib_err;
        bool near_self = fabs(chi - Tme) <= chi_err, near_best = false;
        if (mode != kNew) {
          const double e2 = chi_err + eb;
          near_best = fabs(chi - chib * o.one_minus_tau) <= e2 ||
                      fabs(chi - chib * o.one_plus_tau) <= e2 ||
                      fabs(chi - chib * o.one_minus_min_delta) <= e2;
        }
        if (near_self || near_best) {
          S.mode_saved = mode;
          if (near_best && eb > 0.0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              S.cand[q] = pc[q];
              pc[q] = S.best[q];
            }
            mode = kRecheckBest;
          } else {
            mode = kRecheckCand;
          }
          decide = false;
        }
      }
      if (!decide) {
      } else if (mode == kNew) {
        start = true;
      } else {
        const double Chi = chi, chib = S.chi_best;
        if (mode == kTrialFirst && Chi < chib * o.one_minus_tau) --k;  // improved: less damping
        const bool worse = chib * o.one_plus_tau < Chi;
        if (!small && worse && k < o.lambda_max_exp10) {
          ++k;  // more damping, retry from best
          mode = kTrialRetry;
          do_solve = true;
        } else if (worse || __builtin_isnan(Chi)) {
          status = SPOTFIT_NOT_CONVERGED;
          out_best = true;
          done = true;
        } else if (Chi < Tme) {
          status = SPOTFIT_MAX_ERROR;
          done = true;
        } else if (chib * o.one_minus_min_delta < Chi) {
          status = SPOTFIT_MIN_DELTA;
          done = true;
        } else if (small) {
          status = SPOTFIT_MIN_STEP;
          done = true;
        } else {
          start = true;
        }
      }
      if (start) {  // a new iteration at the accepted point pc
        if (it >= o.max_iter) {
          status = SPOTFIT_MAX_ITER;
          done = true;
        } else {
          ++it;
          ++n_grad;
          if (__builtin_isnan(chi)) {
            status = SPOTFIT_NOT_CONVERGED;
            done = true;
          } else if (chi < Tme) {
            status = SPOTFIT_MAX_ERROR;
            done = true;
          } else {
            S.chi_best = chi;
            S.chib_err = chi_err;
            S.a_best = a;
            S.b_best = b;
#pragma unroll
            for (int q = 0; q < 4; ++q) S.best[q] = pc[q];
            mode = kTrialFirst;
            do_grad = true;
            do_solve = true;
          }
        }
      }

      // ================= results and the next spot =================
      if (done) {
        if (li == 0) {
          float* po = ka.params_out + 6 * s;
          if (out_best) {
            po[0] = float(S.best[0]);
            po[1] = float(S.best[1]);
            po[2] = float(S.best[2]);
            po[3] = float(S.best[3]);
            po[4] = float(S.a_best);
            po[5] = float(S.b_best);
            ka.chi2_out[s] = float(S.chi_best);
          } else {
            po[0] = float(pc[0]);
            po[1] = float(pc[1]);
            po[2] = float(pc[2]);
            po[3] = float(pc[3]);
            po[4] = float(a);
            po[5] = float(b);
            ka.chi2_out[s] = float(chi);
          }
          ka.iters_out[s] = it;
          ka.status_out[s] = status;
          if (ka.evals_out) {
            ka.evals_out[2 * s] = n_grad;
            ka.evals_out[2 * s + 1] = n_trial;
          }
        }
        advance();
        took = true;
      }

      // pixels for the next step's evaluation (the next spot's after a take), issued
      // before the derivative pass and the solve so that those cover their latency
      if (s >= 0) load_pixels();

      // ================= derivative pass at pc (Eqs. 7-9, 11) =================
      if (do_grad) {
        const double x = pc[0], y = pc[1];
        // moments of the lane's columns and rows
        double v[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) v[q] = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const int c = li + L * j;
          const double dx = double(c) - x, dy = double(c) - y;
          const double ex2 = ex[j] * ex[j], ey2 = eyl[j] * eyl[j];
          const double dx2 = dx * dx, dy2 = dy * dy;
          v[0] = __builtin_fma(dx, ex[j], v[0]);
          v[1] = __builtin_fma(dx2, ex[j], v[1]);
          v[2] = __builtin_fma(dx, ex2, v[2]);
          v[3] = __builtin_fma(dx2, ex2, v[3]);
          v[4] = __builtin_fma(dx2 * dx, ex2, v[4]);
          v[5] = __builtin_fma(dx2 * dx2, ex2, v[5]);
          v[6] = __builtin_fma(dy, eyl[j], v[6]);
          v[7] = __builtin_fma(dy2, eyl[j], v[7]);
          v[8] = __builtin_fma(dy, ey2, v[8]);
          v[9] = __builtin_fma(dy2, ey2, v[9]);
          v[10] = __builtin_fma(dy2 * dy, ey2, v[10]);
          v[11] = __builtin_fma(dy2 * dy2, ey2, v[11]);
        }
#pragma unroll
        for (int q = 0; q < 12; ++q) v[q] = gsum<L>(v[q]);
        // X[k] = sum dx^k ex (k < 3), Xq[k] = sum dx^k ex^2 (k < 5); same for rows
        const double Sx = S.Sx, Sxx = S.Sxx, Sy = S.Sy, Syy = S.Syy, FG = S.FG;
        const double X[3] = {Sx, v[0], v[1]};
        const double Xq[5] = {Sxx, v[2], v[3], v[4], v[5]};
        const double Y[3] = {Sy, v[6], v[7]};
        const double Yq[5] = {Syy, v[8], v[9], v[10], v[11]};
        const double Bj[4] = {S.Bx, S.By, S.Bsx, S.Bsy};  // sum g d_j f / w_j for x, y, sx, sy
        const double isx = rcp_nr(pc[2]), isy = rcp_nr(pc[3]);
        const double Nn = double(w * h), iD = rcp_nr(S.D);
        const double F = Sx * Sy, FF = Sxx * Syy;
        const double wt[4] = {isx * isx, isy * isy, isx * isx * isx, isy * isy * isy};
        // Eq. 7 sums of parameter j, Eq. 8 amplitude derivatives, and the right-hand
        // side; the normal matrix, with J_j = da_j f + a df_j + db_j (Eq. 9, second
        // factor), is
        //   sum J_i J_j = da_i W_j + db_i Z_j + a (da_j Sfd_i + db_j dF_i) + a^2 sum df_i df_j
        // with W_j = da_j FF + a Sfd_j + db_j F and Z_j = da_j F + a dF_j + N db_j
        const double sfr = a * FF + b * F - FG;  // sum f r  (0 up to rounding, Eq. 4)
        const double sr = a * F + b * Nn - Gs;   // sum r
        double da[4], db[4], W[4], Z[4], aS[4], aF[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int ox = ox_of(j), oy = oy_of(j);
          const double dF = X[ox] * Y[oy] * wt[j];
          const double Sfd = Xq[ox] * Yq[oy] * wt[j];
          const double dFG = Bj[j] * wt[j];
          const double dFF = 2.0 * Sfd;
          const double gam = Nn * dFF - 2.0 * F * dF;
          da[j] = (Nn * dFG - Gs * dF - a * gam) * iD;
          db[j] = (Gs * dFF - FG * dF - F * dFG - b * gam) * iD;
          aS[j] = a * Sfd;
          aF[j] = a * dF;
          W[j] = __builtin_fma(da[j], FF, __builtin_fma(db[j], F, aS[j]));
          Z[j] = __builtin_fma(da[j], F, __builtin_fma(db[j], Nn, aF[j]));
          S.bv[j] = -(da[j] * sfr + a * (a * Sfd + b * dF - dFG) + db[j] * sr);
        }
        const double a2 = a * a;
#pragma unroll
        for (int t = 0; t < 10; ++t) {
          const int i = tri_i(t), j = tri_j(t);
          const double Sdd = Xq[ox_of(i) + ox_of(j)] * Yq[oy_of(i) + oy_of(j)] * (wt[i] * wt[j]);
          S.A[t] = __builtin_fma(da[i], W[j],
                                 __builtin_fma(db[i], Z[j],
                                               __builtin_fma(da[j], aS[i],
                                                             __builtin_fma(db[j], aF[i], a2 * Sdd))));
        }
        if (sym) {  // sigma = sx = sy: contract along d/dsigma = d/dsx + d/dsy, pad with identity
          S.A[2] += S.A[3];
          S.A[3] = 0.0;
          S.A[5] += S.A[6];
          S.A[6] = 0.0;
          S.A[7] += 2.0 * S.A[8] + S.A[9];
          S.A[8] = 0.0;
          // 1.0 made here: held across the loop instead, it is a register the
          // allocator spills when the mixed launch inlines three class loops
          double one;
          asm volatile("v_mov_b64 %0, 1.0" : "=v"(one));
          S.A[9] = one;
          S.bv[2] += S.bv[3];
          S.bv[3] = 0.0;
        }
      }

      // ================= damped step (Eq. 14) and limit() =================
      if (do_solve) {
        double d[4];
        solve4(S.A, S.bv, pow10i(k), d);
        const double smax = o.sigma_max_frac * double(w > h ? w : h);
        const double b0 = S.best[0], b1 = S.best[1], b2 = S.best[2], b3 = S.best[3];
        const double p2 = clampn(b2 + d[2], o.sigma_min, smax);
        pc[0] = clampn(b0 + d[0], -0.5, double(w) - 0.5);
        pc[1] = clampn(b1 + d[1], -0.5, double(h) - 0.5);
        pc[2] = p2;
        pc[3] = sym ? p2 : clampn(b3 + d[3], o.sigma_min, smax);
        // MinStep: every step below min_step_rel of its parameter, the centre
        // measured from the centre of the ROI
        small = fabs(d[0]) < o.min_step_rel * fabs(b0 - 0.5 * double(w - 1)) &&
                fabs(d[1]) < o.min_step_rel * fabs(b1 - 0.5 * double(h - 1)) &&
                fabs(d[2]) < o.min_step_rel * fabs(b2) &&
                (sym || fabs(d[3]) < o.min_step_rel * fabs(b3));
      }

    }
    reserve(took);
  }
}

template <int L, int CPL, int WPE, int DT, bool RAW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_narrow_kernel(KArgs ka) {
  __shared__ NState sts[64 / L];
  __shared__ float4 cinit[RAW ? 2 * (64 / L) : 1];
  fit_narrow<L, CPL, DT, RAW>(ka, SpotQueue{nullptr, ka.queue, (int32_t)ka.n}, sts, cinit);
}

// Batches of uneven spot sizes: the classify pass of the wide kernel's mixed
// launch buckets spots by size class; each wavefront runs the plan of one class
// and moves on to the next class when that class's list runs dry.
template <int L0, int C0, int L1, int C1, int L2, int C2, int WPE, int DT, bool RAW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_narrow_mixed_kernel(
    KArgs ka, MixedWs ws) {
  __shared__ NState sts[64 / L0];
  __shared__ float4 cinit[RAW ? 2 * (64 / L0) : 1];
  static_assert(L0 <= L1 && L1 <= L2, "classes in order of size");
  const int start = blockIdx.x % 3;
  for (int q = 0; q < 3; ++q) {
    const int c = (start + q) % 3;
    const int32_t* list = ws.lists + (int64_t)c * ws.cap;
    int32_t* take = ws.counters + 3 + c;
    const int32_t count = ws.counters[c];
    if (c == 0)
      fit_narrow<L0, C0, DT, RAW>(ka, SpotQueue{list, take, count}, sts, cinit);
    else if (c == 1)
      fit_narrow<L1, C1, DT, RAW>(ka, SpotQueue{list, take, count}, sts, cinit);
    else
      fit_narrow<L2, C2, DT, RAW>(ka, SpotQueue{list, take, count}, sts, cinit);
  }
}

// Whether the lane-owned classes of a mixed-size launch skip the passes of
// empty slots: not taken, since a wavefront's last spots of one class overlap
// the other wavefronts' spots of the next (skipping measured 0.8 % slower on
// 2M spots of sides 7..32).
constexpr bool kMixedSkip = false;

// A mixed-size launch whose <= 16 px class runs the lane-owned mapping (4-lane
// groups of 4 spots, CPL1 columns per lane), and with OWN2 > 0 its <= 32 px
// class too (L2-lane groups of OWN2 spots); a launch that computes its start
// values runs the narrow mappings of the same widths instead.  The classes run
// one after another, so their LDS state shares one region.
template <int L0, int C0, int CPL1, int L2, int C2, int OWN2, int WPE, int DT, bool RAW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void fit_owned_mixed_kernel(
    KArgs ka, MixedWs ws) {
  static_assert(L0 <= 4 && 4 <= L2, "classes in order of size");
  struct Narrow {
    NState sts[64 / L0];
    float4 cinit[RAW ? 2 * (64 / L0) : 1];
  };
  __shared__ union Lds {
    Narrow n;
    own::OShared o;
  } lds;
  const int start = blockIdx.x % 3;
  for (int q = 0; q < 3; ++q) {
    const int c = (start + q) % 3;
    const int32_t* list = ws.lists + (int64_t)c * ws.cap;
    int32_t* take = ws.counters + 3 + c;
    const int32_t count = ws.counters[c];
    if (c == 0) {
      fit_narrow<L0, C0, DT, RAW>(ka, SpotQueue{list, take, count}, lds.n.sts, lds.n.cinit);
    } else if (c == 1) {
      if constexpr (RAW)
        fit_narrow<4, CPL1, DT, RAW>(ka, SpotQueue{list, take, count}, lds.n.sts, lds.n.cinit);
      else
        own::fit_owned<4, CPL1, DT, 4, kMixedSkip>(ka, list, take, count, lds.o);
    } else {
      if constexpr (OWN2 > 0 && !RAW)
        own::fit_owned<L2, C2, DT, OWN2, kMixedSkip>(ka, list, take, count, lds.o);
      else
        fit_narrow<L2, C2, DT, RAW>(ka, SpotQueue{list, take, count}, lds.n.sts, lds.n.cinit);
    }
  }
}

}  // namespace nrw

// The compiled narrow plans: (lanes per spot, columns per lane, min waves per SIMD).
#define SF_NARROW_PLANS(X) \
  X(0, 4, 2, 2)            \
  X(1, 4, 4, 2)            \
  X(2, 8, 2, 2)            \
  X(3, 16, 2, 2)

int narrow_plan_count() { return 4; }

void narrow_plan_shape(int plan, int* lanes, int* cpl) {
#define SF_NSHAPE(I, L, C, W) \
  if (plan == I) {            \
    *lanes = L;               \
    *cpl = C;                 \
    return;                   \
  }
  SF_NARROW_PLANS(SF_NSHAPE)
#undef SF_NSHAPE
  *lanes = 0;
  *cpl = 0;
}

const void* narrow_kernel_symbol(int plan) {
#define SF_NSYM(I, L, C, W) \
  if (plan == I) return reinterpret_cast<const void*>(&nrw::fit_narrow_kernel<L, C, W, SPOTFIT_U16, false>);
  SF_NARROW_PLANS(SF_NSYM)
#undef SF_NSYM
  return nullptr;
}

// Mixed-size plans (size classes <= 8, <= 16, <= 32 px side): lanes and columns
// per class, min waves per SIMD.
#define SF_NARROW_MIXED_PLANS(X) \
  X(0, 4, 2, 4, 4, 16, 2, 2)       \
  X(1, 4, 2, 8, 2, 16, 2, 2)

// Mixed-size plans whose <= 16 px class is lane-owned: lanes and columns of
// class 0, columns per lane of class 1, lanes and columns of class 2, spots per
// group of class 2 (0: narrow), min waves per SIMD.
#define SF_OWNED_MIXED_PLANS(X) X(2, 4, 2, 4, 16, 2, 0, 2) X(3, 4, 2, 4, 16, 2, 4, 2)

int narrow_mixed_plan_count() { return 4; }

const void* narrow_mixed_kernel_symbol(int plan) {
#define SF_OMSYM(I, A, B, C, D, E, O, W) \
  if (plan == I)                         \
    return reinterpret_cast<const void*>(&nrw::fit_owned_mixed_kernel<A, B, C, D, E, O, W, SPOTFIT_U16, false>);
  SF_OWNED_MIXED_PLANS(SF_OMSYM)
#undef SF_OMSYM
#define SF_NMSYM(I, A, B, C, D, E, F, W) \
  if (plan == I)                         \
    return reinterpret_cast<const void*>(&nrw::fit_narrow_mixed_kernel<A, B, C, D, E, F, W, SPOTFIT_U16, false>);
  SF_NARROW_MIXED_PLANS(SF_NMSYM)
#undef SF_NMSYM
  return nullptr;
}

hipError_t launch_narrow_mixed_fit(int plan, const KArgs& ka, const MixedWs& ws, int grid,
                                   hipStream_t st) {
  const bool raw = ka.init_out != nullptr;
#define SF_NMLAUNCH(I, A, B, C, D, E, F, W)                                                     \
  if (plan == I) {                                                                              \
    if (ka.dtype == SPOTFIT_U16 && raw)                                                         \
      hipLaunchKernelGGL((nrw::fit_narrow_mixed_kernel<A, B, C, D, E, F, W, SPOTFIT_U16, true>), \
                         dim3(grid), dim3(64), 0, st, ka, ws);                                  \
    else if (ka.dtype == SPOTFIT_U16)                                                           \
      hipLaunchKernelGGL((nrw::fit_narrow_mixed_kernel<A, B, C, D, E, F, W, SPOTFIT_U16, false>), \
                         dim3(grid), dim3(64), 0, st, ka, ws);                                  \
    else if (raw)                                                                               \
      hipLaunchKernelGGL((nrw::fit_narrow_mixed_kernel<A, B, C, D, E, F, W, SPOTFIT_F32, true>), \
                         dim3(grid), dim3(64), 0, st, ka, ws);                                  \
    else                                                                                        \
      hipLaunchKernelGGL((nrw::fit_narrow_mixed_kernel<A, B, C, D, E, F, W, SPOTFIT_F32, false>), \
                         dim3(grid), dim3(64), 0, st, ka, ws);                                  \
    return hipGetLastError();                                                                 \
  }
  SF_NARROW_MIXED_PLANS(SF_NMLAUNCH)
#undef SF_NMLAUNCH
#define SF_OMLAUNCH(I, A, B, C, D, E, O, W)                                                      \
  if (plan == I) {                                                                               \
    if (ka.dtype == SPOTFIT_U16 && raw)                                                          \
      hipLaunchKernelGGL((nrw::fit_owned_mixed_kernel<A, B, C, D, E, O, W, SPOTFIT_U16, true>), dim3(grid), \
                         dim3(64), 0, st, ka, ws);                                               \
    else if (ka.dtype == SPOTFIT_U16)                                                            \
      hipLaunchKernelGGL((nrw::fit_owned_mixed_kernel<A, B, C, D, E, O, W, SPOTFIT_U16, false>), dim3(grid), \
                         dim3(64), 0, st, ka, ws);                                               \
    else if (raw)                                                                                \
      hipLaunchKernelGGL((nrw::fit_owned_mixed_kernel<A, B, C, D, E, O, W, SPOTFIT_F32, true>), dim3(grid), \
                         dim3(64), 0, st, ka, ws);                                               \
    else                                                                                         \
      hipLaunchKernelGGL((nrw::fit_owned_mixed_kernel<A, B, C, D, E, O, W, SPOTFIT_F32, false>), dim3(grid), \
                         dim3(64), 0, st, ka, ws);                                               \
    return hipGetLastError();                                                                    \
  }
  SF_OWNED_MIXED_PLANS(SF_OMLAUNCH)
#undef SF_OMLAUNCH
  return hipErrorInvalidValue;
}

__global__ void queue_reset_kernel(int32_t* take) {
  if (threadIdx.x == 0) *take = 0;
}

hipError_t launch_narrow_kernel(int plan, const KArgs& ka, int grid, hipStream_t st) {
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, ka.queue);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool raw = ka.init_out != nullptr;
#define SF_NLAUNCH(I, L, C, W)                                                                      \
  if (plan == I) {                                                                                  \
    if (ka.dtype == SPOTFIT_U16 && raw)                                                             \
      hipLaunchKernelGGL((nrw::fit_narrow_kernel<L, C, W, SPOTFIT_U16, true>), dim3(grid), dim3(64), \
                         0, st, ka);                                                                \
    else if (ka.dtype == SPOTFIT_U16)                                                               \
      hipLaunchKernelGGL((nrw::fit_narrow_kernel<L, C, W, SPOTFIT_U16, false>), dim3(grid),          \
                         dim3(64), 0, st, ka);                                                      \
    else if (raw)                                                                                   \
      hipLaunchKernelGGL((nrw::fit_narrow_kernel<L, C, W, SPOTFIT_F32, true>), dim3(grid), dim3(64), \
                         0, st, ka);                                                                \
    else                                                                                            \
      hipLaunchKernelGGL((nrw::fit_narrow_kernel<L, C, W, SPOTFIT_F32, false>), dim3(grid),          \
                         dim3(64), 0, st, ka);                                                      \
    return hipGetLastError();                                                                      \
  }
  SF_NARROW_PLANS(SF_NLAUNCH)
#undef SF_NLAUNCH
  return hipErrorInvalidValue;
}

}  // namespace sf
