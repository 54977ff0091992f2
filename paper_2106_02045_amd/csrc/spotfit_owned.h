// spotfit_owned.h -- the lane-owned mapping of the batched implicit-amplitude
// Levenberg-Marquardt Gaussian-spot fit on gfx950 (separable form, one spot
// per lane), used by the lane-owned kernel and by the mixed-size launch.
//
// The arithmetic is the narrow kernel's, operation for operation, so the
// results are bitwise the same; the mapping differs.  A group of L lanes (4
// or 16) holds L spots, spot i owned by the group's lane i, and a wavefront 64
// spots (or OWN < L spots per group, each owned by L / OWN lanes):
//
//  * Each wave step makes L passes.  In pass i the whole group evaluates the
//    spot of its lane i at that lane's candidate point, exactly as the narrow
//    kernel's group evaluates its one spot: lane l owns the columns c = l + L*j
//    and their column factors, the row factors of the rows r = l + L*j, and the
//    pixels of its columns (in registers); butterflies give every lane the
//    group totals, and lane i writes them to its slots in LDS.  The pass also
//    forms the one-dimensional moments of the derivative sums (Eqs. 7-9),
//    which the step uses when the point is accepted.
//  * Then every lane takes the scalar steps of its own spot: amplitudes and
//    chi^2 (Eqs. 2, 6), the decisions of the Fit2DGaussian loop, the normal
//    equations (Eq. 9) and the damped solve (Eq. 14) with limit().  The narrow
//    kernel takes these on all L lanes of a group for one spot; here each is
//    taken once per spot, by the lane that owns it.
//  * Pixels: while a pass goes through the rows of its spot, it loads the same
//    rows of the next pass's spot into the registers it is done with.  The
//    first pass's pixels are loaded after the decisions of the step before,
//    ahead of the normal equations and the solve.  A pass whose spot needs
//    chi^2 summed directly (float data, or a close decision re-taken) keeps
//    its pixels for that second sum and loads the next spot's after it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "lanegroup.h"
#include "spotfit_lm.h"
#include "separable.h"

namespace sf {
namespace own {

using namespace lm;
using namespace lg;
using namespace sep;

// Zeros read in place of the columns outside a spot (one row offset of a
// 32 x 32 spot at most).  Never written; not const (see the narrow kernel:
// a constant-memory pointer would turn the pixel loads into FLAT loads).
static __device__ float kZeros[32 * 32];

// Group totals of a pass that its spot's lane keeps: the evaluation sums, the
// twelve derivative moments, and chi^2 summed over the pixels when needed.
enum : int {
  kSx = 0, kSxx, kSy, kSyy, kFG, kBx, kBsx, kR1, kR2,
  kMom,                 // kMom + q, q < 12: the moments v[q] of the derivative pass
  kChiDirect = kMom + 12,
  kSums
};

// LDS of a wavefront (a workgroup is one wavefront): one slot per lane in
// each array, lanes contiguous.
struct OShared {
  double sum[kSums][64];  // the totals of the lane's spot from this step's pass
  double best[4][64];     // point at the start of the iteration
  double chi_best[64], a_best[64], b_best[64];
  double chib_err[64];    // error bound of chi_best (0: summed directly)
  double cand[4][64];     // the candidate while the best point is re-evaluated
  int mode_saved[64];     // the mode whose decision a re-evaluation completes
  // the lane's reserved next spot: start values, pixel offset, shape
  float4 nx_in[64];
  int64_t nx_off[64];
  spotfit_shape_t nx_sh[64];
};

// Where a spot's pixels are: the top of each of the lane's columns (the zero
// block for columns outside the spot) and the row offsets in bytes.
template <int CPL>
struct Src {
  const char* cp[CPL];
  uint32_t step, last;
};

template <int L, int CPL, int DT>
__device__ __forceinline__ Src<CPL> spot_src(const KArgs& ka, int li, int w, int h, int64_t off) {
  constexpr uint32_t esz = DT == SPOTFIT_U16 ? 2u : 4u;
  Src<CPL> s;
  const char* zero = reinterpret_cast<const char*>(kZeros);
#pragma unroll
  for (int j = 0; j < CPL; ++j)
    s.cp[j] = li + L * j < w ? static_cast<const char*>(ka.data) + (off + li + L * j) * esz : zero;
  const int hh = h > 0 ? h : 1;
  s.step = esz * uint32_t(w);
  s.last = uint32_t(hh - 1) * s.step;
  return s;
}

// Row of a spot at byte offset rb (at most the last row's) into ring slot q.
template <int CPL, int W, int DT>
__device__ __forceinline__ void load_row(uint32_t (&g)[CPL][W], int q, const Src<CPL>& s, uint32_t rb) {
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    if constexpr (DT == SPOTFIT_U16)
      g[j][q] = *reinterpret_cast<const uint16_t*>(s.cp[j] + rb);
    else
      g[j][q] = *reinterpret_cast<const uint32_t*>(s.cp[j] + rb);
  }
}

// The first W rows of a spot into the ring (rows below the spot repeat its
// last row; the passes skip them).
template <int CPL, int W, int DT>
__device__ __forceinline__ void load_head(uint32_t (&g)[CPL][W], const Src<CPL>& s) {
  uint32_t rb = 0;
#pragma unroll
  for (int r = 0; r < W; ++r) {
    if (r > 0) rb = __builtin_elementwise_min(rb + s.step, s.last);
    load_row<CPL, W, DT>(g, r, s, rb);
  }
}

// Value of in-group lane p on every lane (the whole wavefront active).
__device__ __forceinline__ int from_lane(int v, int addr) { return __builtin_amdgcn_ds_bpermute(addr, v); }
__device__ __forceinline__ double from_lane(double v, int addr) {
  int2 u = *reinterpret_cast<int2*>(&v);
  int2 r = make_int2(from_lane(u.x, addr), from_lane(u.y, addr));
  return *reinterpret_cast<double*>(&r);
}

// Fit every spot a queue hands to this wavefront: queue position i
// (0 <= i < count) is spot list[i], or spot i itself when list is null; the
// wavefront takes positions from the counter `take` a chunk of 64 at a time.
// L lanes per group, CPL columns per lane: spots with w, h <= L * CPL; pixel
// data type DT.  OWN spots per group: each spot is owned by L / OWN lanes,
// which take its scalar steps alike (OWN = L: one lane per spot).  SKIP: a
// step runs only the passes of slots that hold a spot in some group.
template <int L, int CPL, int DT, int OWN = L, bool SKIP = true>
__device__ __forceinline__ void fit_owned(const KArgs& ka, const int32_t* list, int32_t* take,
                                          int32_t count, OShared& S) {
  static_assert((L == 4 || L == 16) && L % OWN == 0 && OWN >= 2, "lanes and spots per group");
  constexpr int HM = L * CPL;
  constexpr int SH = L / OWN;  // lanes per spot
  const int lane = __lane_id();
  const int li = lane % L;
  const int slot = li / SH;         // the lane's spot in its group
  const bool lead = li % SH == 0;   // the lane that writes the spot's results
  const int gaddr = (lane & ~(L - 1)) << 2;  // ds_bpermute address of the group's lane 0
  const KOpts o = ka.opt;

  // the lane's own spot
  int64_t s = -1;
  int w = 0, h = 0, k = 0, it = 0, mode = kNew, n_trial = 0;  // it: also the derivative passes
  bool bad = false;  // the spot is unusable: it ends at its first step as BAD_INPUT
  bool sym = true, small = false;
  double pc[4] = {0.0, 0.0, 0.0, 0.0};  // candidate point (accepted point after a decision)
  double a = 0.0, b = 0.0, chi = 0.0;   // Eq. 6 amplitudes and Eq. 2 error at pc
  double Gs = 0.0;
  double Vs = 0.0;       // 16-bit data: N sum g^2 - G^2 of the spot (exact)
  double chi_err = 0.0;  // bound on |chi - chi summed over the pixels|
  double A[10], bv[4];   // normal equations at best (upper triangle), kept for retries
#pragma unroll
  for (int t = 0; t < 10; ++t) A[t] = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) bv[j] = 0.0;
  int64_t off = 0;  // element offset of the spot's pixels

  // Pixels of the lane's columns (0 outside the spot): a ring of W rows.  A
  // loop over a spot's rows finds its first W rows loaded; after using row r it
  // loads row r + W into the same slot, and in its last W rows the head of the
  // next loop's spot (the tail source), so that a load is used W rows after it
  // is issued and only W rows take registers.
  constexpr int W = L == 16 ? 8 : 4;  // 16-lane groups: 32 rows, loads further ahead
  static_assert(HM % W == 0, "ring rows");
  uint32_t g[CPL][W];
  auto row_loop = [&](const double (&eyl)[CPL], int hs, const Src<CPL>& cur, const Src<CPL>& tail,
                      auto body) {
    uint32_t rbc = __builtin_elementwise_min(uint32_t(W) * cur.step, cur.last), rbt = 0;
    for_rows<L, CPL, HM>(eyl, [&](int r, double e) {
      if (r < hs) body(r, e, r % W);
      if (r + W < HM) {
        if (r > 0) rbc = __builtin_elementwise_min(rbc + cur.step, cur.last);
        load_row<CPL, W, DT>(g, r % W, cur, rbc);
      } else {  // every slot is loaded (from the zero block when there is no tail), so
                // that no slot keeps an older value
        if (r + W > HM) rbt = __builtin_elementwise_min(rbt + tail.step, tail.last);
        load_row<CPL, W, DT>(g, r % W, tail, rbt);
      }
    });
  };

  // The next spot, reserved one ahead, with its description already loaded
  // (into the lane's slots in LDS).
  int32_t ns = -1;

  // Queue positions: the wavefront's chunk [cbase, cbase + 64) of which cused
  // are handed out, and the next chunk, requested from the counter once half
  // of the current one is out.
  constexpr int kChunk = 64 / SH;
  int cbase = 0, cused = 0, nbase_l0 = 0;
  bool nb_asked = false;
  {
    int b0 = 0;
    if (lane == 0) b0 = atomicAdd(take, kChunk);
    cbase = __builtin_amdgcn_readfirstlane(b0);
  }
  // Give every lane with `want` a new reserved spot (whole wavefront active).
  auto reserve = [&](bool want) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(want && lead);
    const int nreq = __builtin_popcountll(m);
    if (nreq == 0) return;
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    int pos;
    if (cused + nreq > kChunk) {  // nreq <= 64: the rest comes from the next chunk
      if (!nb_asked && lane == 0) nbase_l0 = atomicAdd(take, kChunk);
      const int nb = __builtin_amdgcn_readfirstlane(nbase_l0);
      pos = cused + rank < kChunk ? cbase + cused + rank : nb + (cused + rank - kChunk);
      cbase = nb;
      cused = cused + nreq - kChunk;
      nb_asked = false;
    } else {
      pos = cbase + cused + rank;
      cused += nreq;
    }
    if (!nb_asked && 2 * cused >= kChunk) {
      if (lane == 0) nbase_l0 = atomicAdd(take, kChunk);
      nb_asked = true;
    }
    if (want && lead) ns = (uint32_t)pos < (uint32_t)count ? (list ? list[pos] : pos) : -1;
    if constexpr (SH > 1) ns = from_lane(ns, (lane & ~(SH - 1)) << 2);  // the spot's lanes alike
    if (want) {
      if (ns >= 0) {
        S.nx_sh[lane] = ka.sizes[ns];
        S.nx_off[lane] = ka.offsets[ns];
        const float* in = ka.init + 4 * (int64_t)ns;
        S.nx_in[lane] = make_float4(in[0], in[1], in[2], in[3]);
      }
    }
  };

  // Take the reserved spot; an unusable one is marked and ends at its next
  // step with BAD_INPUT.
  auto advance = [&]() {
    s = ns;
    ns = -1;
    if (s < 0) return;
    const spotfit_shape_t sh = S.nx_sh[lane];
    const float4 nin = S.nx_in[lane];
    const float i0 = nin.x, i1 = nin.y, i2 = nin.z, i3 = nin.w;
    off = S.nx_off[lane];
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
    k = o.lambda0_exp10;
    it = 0;
    mode = kNew;
    n_trial = 0;
  };

  // the pixels of the group's spot p
  auto src_of = [&](int p) {
    const int addr = gaddr + ((p * SH) << 2);
    const int wv = s >= 0 ? w : 0, hv = s >= 0 ? h : 0;
    const int ws = from_lane(wv, addr), hs = from_lane(hv, addr);
    const int64_t os = (int64_t)(((uint64_t)(uint32_t)from_lane((int)(uint32_t)off, addr)) |
                                 ((uint64_t)(uint32_t)from_lane((int)(off >> 32), addr) << 32));
    return spot_src<L, CPL, DT>(ka, li, ws, hs, os);
  };

  // no pixels: every column reads the zero block
  const Src<CPL> none = spot_src<L, CPL, DT>(ka, li, 0, 0, 0);

  // The passes of a step: one per slot that holds a spot in some group, in slot
  // order, packed 4 bits each (as a wavefront's spots run out, its steps skip
  // the slots that no group uses).
  constexpr uint64_t kSlot0 = [] {
    uint64_t m = 0;
    for (int gi = 0; gi < 64 / L; ++gi) m |= uint64_t(1) << (gi * L);
    return m;
  }();
  int npass = 0;
  auto pass_order = [&]() -> uint32_t {
    const uint64_t lv = __builtin_amdgcn_ballot_w64(s >= 0 && lead);
    uint32_t ord = 0;
    int n = 0;
#pragma unroll
    for (int p = 0; p < OWN; ++p) {
      if (!SKIP || (lv & (kSlot0 << (p * SH)))) {
        ord |= uint32_t(p) << (4 * n);
        ++n;
      }
    }
    npass = n;
    return ord;
  };

  reserve(true);
  advance();
  reserve(true);
  uint32_t ord = pass_order();
  load_head<CPL, W, DT>(g, src_of(int(ord & 15u)));

  while (__builtin_amdgcn_ballot_w64(s >= 0) != 0) {
    const int wv = s >= 0 ? w : 0, hv = s >= 0 ? h : 0;
    // chi^2 summed over the pixels: always for float data, for 16-bit data only
    // where a close decision is being re-taken
    const bool dir_own = s >= 0 && !bad &&
                         (DT != SPOTFIT_U16 || mode == kRecheckBest || mode == kRecheckCand);

    // ================= passes: the group evaluates each of its spots =================
#pragma unroll 1
    for (int i = 0; i < npass; ++i) {
      const int p = int((ord >> (4 * i)) & 15u);
      const int addr = gaddr + ((p * SH) << 2);
      const bool mine = slot == p;
      const int ws = from_lane(wv, addr), hs = from_lane(hv, addr);
      const int md = from_lane(mode, addr);
      const bool dr = from_lane((int)dir_own, addr) != 0;
      const double x = from_lane(pc[0], addr), y = from_lane(pc[1], addr);
      const double p2 = from_lane(pc[2], addr), p3 = from_lane(pc[3], addr);
      const double gs_spot = from_lane(Gs, addr);
      const bool more = i + 1 < npass;
      const Src<CPL> cur = src_of(p);
      const Src<CPL> nx = more ? src_of(int((ord >> (4 * i + 4)) & 15u)) : none;

      // trial evaluation at the spot's point (Eqs. 2, 5, 6, 10)
      const double hx = -0.5 * rcp_nr(p2 * p2);
      const double hy = -0.5 * rcp_nr(p3 * p3);
      double ex[CPL], eyl[CPL];
      double sxp = 0.0, sxxp = 0.0, syp = 0.0, syyp = 0.0;
      {
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
          ex[j] = c < ws ? fac[j] : 0.0;
          eyl[j] = c < hs ? fac[CPL + j] : 0.0;
          sxp += ex[j];
          sxxp = __builtin_fma(ex[j], ex[j], sxxp);
          syp += eyl[j];
          syyp = __builtin_fma(eyl[j], eyl[j], syyp);
        }
      }
      // column sums t(c) = sum_r g ey and row sums s(r) = sum_c g ex (lane's
      // columns); the tail loads the next pass's spot, or this spot again when
      // the wavefront sums chi^2 directly in this pass
      const bool any_dr = __builtin_amdgcn_ballot_w64(dr) != 0;
      double t[CPL];
#pragma unroll
      for (int j = 0; j < CPL; ++j) t[j] = 0.0;
      double gp = 0.0, byp = 0.0, bsyp = 0.0, gsum_px = 0.0, ggp = 0.0;
      uint32_t gsi = 0;
      row_loop(eyl, hs, cur, any_dr ? cur : nx, [&](int r, double e, int q) {
        double sr = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const double gd = pixel<DT>(g[j][q]);
          t[j] = __builtin_fma(gd, e, t[j]);
          sr = __builtin_fma(gd, ex[j], sr);
          if constexpr (DT == SPOTFIT_U16) {
            gsi += g[j][q];
            ggp = __builtin_fma(gd, gd, ggp);
          } else {
            gsum_px += gd;
          }
        }
        const double es = e * sr;
        gp += es;
        byp = __builtin_fma(double(r), es, byp);
        bsyp = __builtin_fma(double(r * r), es, bsyp);
      });
      double bxp = 0.0, bsxp = 0.0;
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const double dx = double(li + L * j) - x;
        const double et = ex[j] * t[j];
        bxp = __builtin_fma(dx, et, bxp);
        bsxp = __builtin_fma(dx * dx, et, bsxp);
      }
      const double Nn = double(ws * hs);
      double Gp = gs_spot;
      if (md == kNew) {  // per-spot constants of a new spot
        if constexpr (DT == SPOTFIT_U16) {
          Gp = double(gsum_i<L>((int)gsi));
          const double Vp = Nn * gsum<L>(ggp) - Gp * Gp;  // every step exact
          if (mine) Vs = Vp;
        } else {
          Gp = gsum<L>(gsum_px);
        }
        if (mine) Gs = Gp;
      }
      const double Sx = gsum<L>(sxp), Sxx = gsum<L>(sxxp);
      const double Sy = gsum<L>(syp), Syy = gsum<L>(syyp);
      const double FG = gsum<L>(gp);
      const double Bx = gsum<L>(bxp), Bsx = gsum<L>(bsxp);
      const double R1 = gsum<L>(byp), R2 = gsum<L>(bsyp);  // sum r e s(r), sum r^2 e s(r)
      if (mine) {
        S.sum[kSx][lane] = Sx;
        S.sum[kSxx][lane] = Sxx;
        S.sum[kSy][lane] = Sy;
        S.sum[kSyy][lane] = Syy;
        S.sum[kFG][lane] = FG;
        S.sum[kBx][lane] = Bx;
        S.sum[kBsx][lane] = Bsx;
        S.sum[kR1][lane] = R1;
        S.sum[kR2][lane] = R2;
      }
      // moments of the lane's columns and rows for the derivative sums
      {
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
        if (mine) {
#pragma unroll
          for (int q = 0; q < 12; ++q) S.sum[kMom + q][lane] = v[q];
        }
      }
      if (any_dr) {
        // the residual sum of squares at the amplitudes of Eq. 6, r = alpha f + beta - g
        // (every group runs the loop for its loads; the spots that asked sum)
        const Amplitudes amp = amplitudes(Nn, Sx, Sxx, Sy, Syy, FG, Gp);
        const double ap = amp.a, bp = amp.b;
        double aex[CPL], bm[CPL], c2[CPL];
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          aex[j] = ap * ex[j];
          bm[j] = li + L * j < ws ? bp : 0.0;
          c2[j] = 0.0;
        }
        row_loop(eyl, dr ? hs : 0, cur, nx, [&](int r, double e, int q) {
#pragma unroll
          for (int j = 0; j < CPL; ++j) {
            const double res = __builtin_fma(aex[j], e, bm[j] - pixel<DT>(g[j][q]));
            c2[j] = __builtin_fma(res, res, c2[j]);
          }
        });
        if (dr) {
          double c2s = c2[0];
#pragma unroll
          for (int j = 1; j < CPL; ++j) c2s += c2[j];
          const double cd = gsum<L>(c2s);
          if (mine) S.sum[kChiDirect][lane] = cd;
        }
      }
    }

    // ================= the lane's own spot: chi^2 and decisions =================
    bool took = false, do_grad = false, do_solve = false;
    double Sx = 0.0, Sxx = 0.0, Sy = 0.0, Syy = 0.0, FG = 0.0, D = 0.0;
    double Bx = 0.0, Bsx = 0.0, By = 0.0, Bsy = 0.0;
    if (s >= 0 && bad) {
      if (lead) {
        float* po = ka.params_out + 6 * s;
        const float nanf = __builtin_nanf("");
#pragma unroll
        for (int q2 = 0; q2 < 6; ++q2) po[q2] = nanf;
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
    } else if (s >= 0) {
      Sx = S.sum[kSx][lane];
      Sxx = S.sum[kSxx][lane];
      Sy = S.sum[kSy][lane];
      Syy = S.sum[kSyy][lane];
      FG = S.sum[kFG][lane];
      Bx = S.sum[kBx][lane];
      Bsx = S.sum[kBsx][lane];
      {
        const double y = pc[1];
        const double R1 = S.sum[kR1][lane], R2 = S.sum[kR2][lane];
        By = __builtin_fma(-y, FG, R1);                                 // sum (r - y) e s(r)
        Bsy = __builtin_fma(-y, __builtin_fma(2.0, R1, -y * FG), R2);  // sum (r - y)^2 e s(r)
      }
      const double Nn = double(w * h);
      const Amplitudes am = amplitudes(Nn, Sx, Sxx, Sy, Syy, FG, Gs);
      D = am.D;
      const bool okD = D > 0.0 && __builtin_isfinite(D);
      a = am.a;
      b = am.b;
      if constexpr (DT == SPOTFIT_U16) chi_closed(Vs, am, Nn, FG, Gs, w, h, chi, chi_err);  // Eq. 2
      if (dir_own) {
        chi = S.sum[kChiDirect][lane];
        chi_err = 0.0;
      }
      if (!okD || !__builtin_isfinite(chi) || !__builtin_isfinite(a) || !__builtin_isfinite(b))
        chi = __builtin_nan("");
      if (mode == kTrialFirst || mode == kTrialRetry) ++n_trial;
      const double Tme = o.max_error_per_px * Nn;
      int status = SPOTFIT_MAX_ITER;

      bool start = false, done = false, out_best = false;
      bool decide = true;
      if (mode == kRecheckBest) {
        // the best point's chi^2, summed directly; then the candidate's
        S.chi_best[lane] = chi;
        S.chib_err[lane] = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) pc[q] = S.cand[q][lane];
        mode = kRecheckCand;
        decide = false;
      } else if (mode == kRecheckCand) {
        mode = S.mode_saved[lane];  // chi is now summed directly: take the decision
      } else if (chi_err > 0.0) {
        // a decision closer to its threshold than the closed form's error bound
        // is re-taken with chi^2 summed directly (the best point's too when that
        // comparison involves it)
        const double chib = S.chi_best[lane], eb = S.chib_err[lane];
        bool near_self = fabs(chi - Tme) <= chi_err, near_best = false;
        if (mode != kNew) {
          const double e2 = chi_err + eb;
          near_best = fabs(chi - chib * o.one_minus_tau) <= e2 ||
                      fabs(chi - chib * o.one_plus_tau) <= e2 ||
                      fabs(chi - chib * o.one_minus_min_delta) <= e2;
        }
        if (near_self || near_best) {
          S.mode_saved[lane] = mode;
          if (near_best && eb > 0.0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              S.cand[q][lane] = pc[q];
              pc[q] = S.best[q][lane];
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
        const double Chi = chi, chib = S.chi_best[lane];
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
          if (__builtin_isnan(chi)) {
            status = SPOTFIT_NOT_CONVERGED;
            done = true;
          } else if (chi < Tme) {
            status = SPOTFIT_MAX_ERROR;
            done = true;
          } else {
            S.chi_best[lane] = chi;
            S.chib_err[lane] = chi_err;
            S.a_best[lane] = a;
            S.b_best[lane] = b;
#pragma unroll
            for (int q = 0; q < 4; ++q) S.best[q][lane] = pc[q];
            mode = kTrialFirst;
            do_grad = true;
            do_solve = true;
          }
        }
      }
      if (done) {
        if (lead) {
          float* po = ka.params_out + 6 * s;
          if (out_best) {
            po[0] = float(S.best[0][lane]);
            po[1] = float(S.best[1][lane]);
            po[2] = float(S.best[2][lane]);
            po[3] = float(S.best[3][lane]);
            po[4] = float(S.a_best[lane]);
            po[5] = float(S.b_best[lane]);
            ka.chi2_out[s] = float(S.chi_best[lane]);
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
            ka.evals_out[2 * s] = it;
            ka.evals_out[2 * s + 1] = n_trial;
          }
        }
        advance();
        took = true;
      }
    }

    // pixels of the next step's first pass (its spot may be new), issued before
    // the normal equations and the solve so that those cover their latency
    ord = pass_order();
    load_head<CPL, W, DT>(g, src_of(int(ord & 15u)));

    // ================= normal equations at pc (Eqs. 7-9, 11) =================
    if (do_grad) {
      double v[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) v[q] = S.sum[kMom + q][lane];
      // X[k] = sum dx^k ex (k < 3), Xq[k] = sum dx^k ex^2 (k < 5); same for rows
      const double X[3] = {Sx, v[0], v[1]};
      const double Xq[5] = {Sxx, v[2], v[3], v[4], v[5]};
      const double Y[3] = {Sy, v[6], v[7]};
      const double Yq[5] = {Syy, v[8], v[9], v[10], v[11]};
      const double Bj[4] = {Bx, By, Bsx, Bsy};  // sum g d_j f / w_j for x, y, sx, sy
      const double isx = rcp_nr(pc[2]), isy = rcp_nr(pc[3]);
      const double Nn = double(w * h), iD = rcp_nr(D);
      const double F = Sx * Sy, FF = Sxx * Syy;
      const double wt[4] = {isx * isx, isy * isy, isx * isx * isx, isy * isy * isy};
      // Eq. 7 sums of parameter j, Eq. 8 amplitude derivatives, and the right-hand
      // side; with J_j = da_j f + a df_j + db_j (Eq. 9, second factor):
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
        bv[j] = -(da[j] * sfr + a * (a * Sfd + b * dF - dFG) + db[j] * sr);
      }
      const double a2 = a * a;
#pragma unroll
      for (int t = 0; t < 10; ++t) {
        const int i = tri_i(t), j = tri_j(t);
        const double Sdd = Xq[ox_of(i) + ox_of(j)] * Yq[oy_of(i) + oy_of(j)] * (wt[i] * wt[j]);
        A[t] = __builtin_fma(da[i], W[j],
                             __builtin_fma(db[i], Z[j],
                                           __builtin_fma(da[j], aS[i],
                                                         __builtin_fma(db[j], aF[i], a2 * Sdd))));
      }
      if (sym) {  // sigma = sx = sy: contract along d/dsigma = d/dsx + d/dsy, pad with identity
        A[2] += A[3];
        A[3] = 0.0;
        A[5] += A[6];
        A[6] = 0.0;
        A[7] += 2.0 * A[8] + A[9];
        A[8] = 0.0;
        A[9] = 1.0;
        bv[2] += bv[3];
        bv[3] = 0.0;
      }
    }

    // ================= damped step (Eq. 14) and limit() =================
    if (do_solve) {
      double d[4];
      solve4(A, bv, pow10i(k), d);
      const double smax = o.sigma_max_frac * double(w > h ? w : h);
      const double b0 = S.best[0][lane], b1 = S.best[1][lane];
      const double b2 = S.best[2][lane], b3 = S.best[3][lane];
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
    reserve(took);
  }
}

}  // namespace own
}  // namespace sf
