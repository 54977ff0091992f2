// spotfit_init.hip -- start values on the device.  The paper takes start
// values as given and leaves them out of its timings (Results section); these
// passes let raw frames go in and fits come out without a host round trip.
//
// The centroid / second-moment estimate (its recipe with the device function
// in spotfit_start.h), and the recipe the paper gives for its accuracy runs
// (Results section): centre = brightest pixel of the 3 x 3 moving average,
// sigma = sqrt(M / pi) with M the pixels above alpha0 exp(-1/2) + beta0.
//
// Mapping: a group of L lanes per spot, lane l owning the columns l + L*j as in
// the fit kernel; groups step over the spots with a grid stride.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lanegroup.h"
#include "spotfit.h"
#include "spotfit_internal.h"
#include "spotfit_start.h"

namespace sf {
namespace ini {

using namespace lg;

template <int L, int CPL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void moment_init_kernel(const void* data, int dtype,
                                                         const spotfit_shape_t* sizes,
                                                         const int64_t* offsets, int64_t n,
                                                         int max_side, int max_pixels,
                                                         float* out) {
  const int lane = __lane_id();
  const int li = lane % L;
  const int64_t stride = (int64_t)gridDim.x * (64 / L);
  // s is the same on every lane of a group, so groups stay whole in the loop
  for (int64_t s = (int64_t)blockIdx.x * (64 / L) + lane / L; s < n; s += stride) {
    const spotfit_shape_t sh = sizes[s];
    if (!usable<L * CPL>(sh, max_side, max_pixels)) {
      if (li == 0) write_nan(out, s);
      continue;
    }
    float o[4];
    moment_init_spot<L, CPL>(data, dtype, sh, offsets[s], li, o);
    if (li == 0)
      for (int q = 0; q < 4; ++q) out[4 * s + q] = o[q];
  }
}

// ---------------------------------------------------------------------------
// The paper's start values.  Per own pixel the 3 x 3 window sum is formed in
// double from the pixel's column and its two neighbours (clamped loads, masked
// outside the ROI) and divided by the number of in-ROI window pixels; the sums
// are exact for 16-bit pixels (and for 32-bit float pixels within 2^26 of each
// other), so their order does not matter.  The group keeps the largest mean
// and, among equal means, the smallest row-major index.
// ---------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ double gmax_d(double v) {
  if constexpr (L >= 2) v = fmax(v, dpp_mov<0xB1>(v));
  if constexpr (L >= 4) v = fmax(v, dpp_mov<0x4E>(v));
  if constexpr (L >= 8) v = fmax(v, dpp_mov<0x141>(v));
  if constexpr (L >= 16) v = fmax(v, dpp_mov<0x140>(v));
  return v;
}

template <int L>
__device__ __forceinline__ float gmin_f(float v) {
  if constexpr (L >= 2) v = fminf(v, dpp_mov<0xB1>(v));
  if constexpr (L >= 4) v = fminf(v, dpp_mov<0x4E>(v));
  if constexpr (L >= 8) v = fminf(v, dpp_mov<0x141>(v));
  if constexpr (L >= 16) v = fminf(v, dpp_mov<0x140>(v));
  return v;
}

template <int L>
__device__ __forceinline__ float gmax_f(float v) {
  if constexpr (L >= 2) v = fmaxf(v, dpp_mov<0xB1>(v));
  if constexpr (L >= 4) v = fmaxf(v, dpp_mov<0x4E>(v));
  if constexpr (L >= 8) v = fmaxf(v, dpp_mov<0x141>(v));
  if constexpr (L >= 16) v = fmaxf(v, dpp_mov<0x140>(v));
  return v;
}

constexpr double kExpMinusHalf = 0x1.368b2fc6f960ap-1;  // e^(-1/2), correctly rounded
constexpr double kPi = 0x1.921fb54442d18p+1;

// Zeros that the loads of a neighbour column outside the spot read instead
// (row offsets of a 32 x 32 spot at most).  Never written; not const, so that
// its pointer and the pixel pointer stay in the global address space.
__device__ uint16_t kZeroCol[32 * 32];

// One butterfly step of the best-window selection: keep the partner's window
// when its mean is larger, or equal with a smaller index.  Both partners see
// the same two windows, so they keep the same one.
template <int CTRL>
__device__ __forceinline__ void best_step(int& bacc, int& bcnt, int& bk) {
  const int pa = dpp_i<CTRL>(bacc), pc = dpp_i<CTRL>(bcnt), pk = dpp_i<CTRL>(bk);
  const int lhs = pa * bcnt, rhs = bacc * pc;
  if (lhs > rhs || (lhs == rhs && pk < bk)) {
    bacc = pa;
    bcnt = pc;
    bk = pk;
  }
}

// 16-bit pixels: the same recipe in integer arithmetic.  A window's sum is an
// integer and its pixel count 4, 6 or 9, so two means compare exactly by cross
// multiplication; for such sums (below 2^20) two different means also differ
// by far more than a double's rounding, so this ordering (and its ties) is the
// one the correctly rounded mean / count quotients give.
template <int L, int CPL>
__device__ __forceinline__ void peak_init_u16(const uint16_t* px, int w, int h, int li, float* o4) {
  int bacc = -1, bcnt = 1, bk = 0x7fffffff;  // best window: sum, pixel count, row-major index
  int lo = 0x7fffffff, hi = -1;
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = li + L * j;
    if (c >= w) continue;
    const uint16_t* cm = c >= 1 ? px + (c - 1) : kZeroCol;
    const uint16_t* cc = px + c;
    const uint16_t* cp = c + 1 < w ? px + (c + 1) : kZeroCol;
    const int ncol = (c >= 1 ? 1 : 0) + 1 + (c + 1 < w ? 1 : 0);
    // rows streamed top to bottom: row sums of the three columns for r - 1, r, r + 1
    int hp = 0;
    int hc = int(cm[0]) + int(cc[0]) + int(cp[0]);
    int gc = int(cc[0]);
#pragma unroll 2
    for (int r = 0; r < h; ++r) {
      int hn = 0, gn = 0;
      if (r + 1 < h) {
        const int ro = (r + 1) * w;
        gn = int(cc[ro]);
        hn = int(cm[ro]) + gn + int(cp[ro]);
      }
      lo = gc < lo ? gc : lo;
      hi = gc > hi ? gc : hi;
      const int acc = hp + hc + hn;
      const int cnt = ncol * ((r >= 1 ? 1 : 0) + 1 + (r + 1 < h ? 1 : 0));
      const int k = r * w + c;
      const int lhs = acc * bcnt, rhs = bacc * cnt;
      if (lhs > rhs || (lhs == rhs && k < bk)) {
        bacc = acc;
        bcnt = cnt;
        bk = k;
      }
      hp = hc;
      hc = hn;
      gc = gn;
    }
  }
  // group: the best window over the lanes (larger mean, then smaller index),
  // and the raw minimum and maximum
  if constexpr (L >= 2) best_step<0xB1>(bacc, bcnt, bk);
  if constexpr (L >= 4) best_step<0x4E>(bacc, bcnt, bk);
  if constexpr (L >= 8) best_step<0x141>(bacc, bcnt, bk);
  if constexpr (L >= 16) best_step<0x140>(bacc, bcnt, bk);
  lo = int(gmin_u<L>(uint32_t(lo)));             // pixel values are >= 0
  hi = 0xffff - int(gmin_u<L>(uint32_t(0xffff - hi)));
  o4[0] = float(bk % w);
  o4[1] = float(bk / w);
  const double beta0 = double(lo), alpha0 = double(hi) - double(lo);
  const double thr = __builtin_fma(alpha0, kExpMinusHalf, beta0);
  int m = 0;
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = li + L * j;
    if (c >= w) continue;
#pragma unroll 4
    for (int r = 0; r < h; ++r) m += double(px[r * w + c]) > thr ? 1 : 0;
  }
  m = gsum_i<L>(m);
  double sig = sqrt(double(m) / kPi);
  sig = sig < 0.5 ? 0.5 : sig;
  o4[2] = o4[3] = float(sig);
}

template <int L, int CPL, int DT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(DT == SPOTFIT_U16 ? 3 : 1))) void
peak_init_kernel(const void* data, int dtype,
                                                       const spotfit_shape_t* sizes,
                                                       const int64_t* offsets, int64_t n,
                                                       int max_side, int max_pixels, float* out) {
  constexpr int HM = L * CPL;
  const int lane = __lane_id();
  const int li = lane % L;
  const int64_t stride = (int64_t)gridDim.x * (64 / L);
  for (int64_t s = (int64_t)blockIdx.x * (64 / L) + lane / L; s < n; s += stride) {
    const spotfit_shape_t sh = sizes[s];
    if (!usable<HM>(sh, max_side, max_pixels)) {
      if (li == 0) write_nan(out, s);
      continue;
    }
    const int w = sh.w, h = sh.h;
    const int64_t off = offsets[s];
    if constexpr (DT == SPOTFIT_U16) {
      float o[4];
      peak_init_u16<L, CPL>(static_cast<const uint16_t*>(data) + off, w, h, li, o);
      if (li == 0)
        for (int q = 0; q < 4; ++q) out[4 * s + q] = o[q];
      continue;
    }
    double best = -__builtin_inf();
    int bk = 0x7fffffff;
    float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int c = li + L * j;
      const bool cin = c < w;
      const int cm = c - 1 < 0 ? 0 : (c - 1 < w ? c - 1 : w - 1);
      const int cc = c < w ? c : w - 1;
      const int cp = c + 1 < w ? c + 1 : w - 1;
      float g0[HM], g1[HM], g2[HM];  // columns c - 1, c, c + 1 (clamped)
#pragma unroll
      for (int r = 0; r < HM; ++r) {
        const int64_t row = off + (int64_t)(r < h ? r : h - 1) * w;
        g0[r] = load_px(data, dtype, row + cm);
        g1[r] = load_px(data, dtype, row + cc);
        g2[r] = load_px(data, dtype, row + cp);
      }
      const bool left = c >= 1, right = c + 1 < w;
      const int ncol = 1 + (left ? 1 : 0) + (right ? 1 : 0);
#pragma unroll
      for (int r = 0; r < HM; ++r) {
        if (!(cin && r < h)) continue;
        double acc = 0.0;
        int nrow = 0;
#pragma unroll
        for (int d = -1; d <= 1; ++d) {
          const int rr = r + d;
          if (rr < 0 || rr >= h) continue;
          ++nrow;
          acc += double(g1[rr]);
          if (left) acc += double(g0[rr]);
          if (right) acc += double(g2[rr]);
        }
        const double mean = acc / double(nrow * ncol);
        const int k = r * w + c;
        if (mean > best || (mean == best && k < bk)) {
          best = mean;
          bk = k;
        }
        lo = fminf(lo, g1[r]);
        hi = fmaxf(hi, g1[r]);
      }
    }
    const double top = gmax_d<L>(best);
    bk = (int)gmin_u<L>(best == top ? (uint32_t)bk : 0xFFFFFFFFu);
    lo = gmin_f<L>(lo);
    hi = gmax_f<L>(hi);
    const double beta0 = double(lo), alpha0 = double(hi) - double(lo);
    const double thr = __builtin_fma(alpha0, kExpMinusHalf, beta0);
    int m = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int c = li + L * j;
      if (c >= w) continue;
#pragma unroll
      for (int r = 0; r < HM; ++r)
        if (r < h) m += double(load_px(data, dtype, off + (int64_t)r * w + c)) > thr ? 1 : 0;
    }
    m = gsum_i<L>(m);
    double sig = sqrt(double(m) / kPi);
    sig = sig < 0.5 ? 0.5 : sig;
    if (li == 0) {
      out[4 * s + 0] = float(bk % w);
      out[4 * s + 1] = float(bk / w);
      out[4 * s + 2] = float(sig);
      out[4 * s + 3] = float(sig);
    }
  }
}

}  // namespace ini

hipError_t launch_start_values(int method, const void* data, int dtype, const spotfit_shape_t* sizes,
                               const int64_t* offsets, int64_t n, int max_side, int max_pixels,
                               float* out, hipStream_t st) {
  // groups of 4 lanes (2 or 4 columns each) up to 16 pixels a side, 16 lanes beyond
  const int cls = max_side <= 8 ? 0 : max_side <= 16 ? 1 : 2;
  const int per_block = cls == 2 ? 4 : 16;
  int64_t blocks = (n + per_block - 1) / per_block;
  blocks = blocks < (1 << 20) ? blocks : (1 << 20);  // the kernels stride over the rest
  const dim3 grid((unsigned)blocks), block(64);
  if (method == kInitMoments) {
    if (cls == 0)
      hipLaunchKernelGGL((ini::moment_init_kernel<4, 2>), grid, block, 0, st, data, dtype, sizes,
                         offsets, n, max_side, max_pixels, out);
    else if (cls == 1)
      hipLaunchKernelGGL((ini::moment_init_kernel<4, 4>), grid, block, 0, st, data, dtype, sizes,
                         offsets, n, max_side, max_pixels, out);
    else
      hipLaunchKernelGGL((ini::moment_init_kernel<16, 2>), grid, block, 0, st, data, dtype, sizes,
                         offsets, n, max_side, max_pixels, out);
  } else if (dtype == SPOTFIT_U16) {
    if (cls == 0)
      hipLaunchKernelGGL((ini::peak_init_kernel<4, 2, SPOTFIT_U16>), grid, block, 0, st, data, dtype,
                         sizes, offsets, n, max_side, max_pixels, out);
    else if (cls == 1)
      hipLaunchKernelGGL((ini::peak_init_kernel<4, 4, SPOTFIT_U16>), grid, block, 0, st, data, dtype,
                         sizes, offsets, n, max_side, max_pixels, out);
    else
      hipLaunchKernelGGL((ini::peak_init_kernel<16, 2, SPOTFIT_U16>), grid, block, 0, st, data, dtype,
                         sizes, offsets, n, max_side, max_pixels, out);
  } else {
    if (cls == 0)
      hipLaunchKernelGGL((ini::peak_init_kernel<4, 2, SPOTFIT_F32>), grid, block, 0, st, data, dtype,
                         sizes, offsets, n, max_side, max_pixels, out);
    else if (cls == 1)
      hipLaunchKernelGGL((ini::peak_init_kernel<4, 4, SPOTFIT_F32>), grid, block, 0, st, data, dtype,
                         sizes, offsets, n, max_side, max_pixels, out);
    else
      hipLaunchKernelGGL((ini::peak_init_kernel<16, 2, SPOTFIT_F32>), grid, block, 0, st, data, dtype,
                         sizes, offsets, n, max_side, max_pixels, out);
  }
  return hipGetLastError();
}

}  // namespace sf
