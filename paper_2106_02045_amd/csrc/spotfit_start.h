// spotfit_start.h -- the centroid / second-moment start values of one spot,
// computed by a group of L lanes (lane l owning the columns l + L*j), as a
// device function shared by the start-value kernel and the fit kernels that
// compute their own start values.
//
// Per spot: background b0 = median of the border ring (top row, bottom row,
// then the left and right columns without the corners; the ring has an even
// number of pixels, so b0 is the mean of its two middle values); weights
// wt = max(g - b0, 0); centre = weighted centroid; var_x = sum wt (x - cx)^2 /
// sum wt (var_y alike); symmetric sigma = sqrt((var_x + var_y) / 2), elliptical
// sigma_x = sqrt(var_x), sigma_y = sqrt(var_y); sigmas clamped to
// [0.8, max(w, h) / 4]; with no positive weight: the ROI centre and sigma 1.5.
//
// The ring median is a radix select, two bits per round, over the 16-bit values
// (or order-preserving 32-bit keys of float values) of the ring pixels, each
// lane holding every L-th of them, so no sort and no LDS are needed; the
// moments are summed in one pass about the ROI centre.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lanegroup.h"
#include "spotfit.h"

namespace sf {
namespace ini {

using namespace lg;

// Order-preserving key of a float (negative values below positive ones).
__device__ __forceinline__ uint32_t key_of(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float value_of(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ float load_px(const void* data, int dtype, int64_t i) {
  return dtype == SPOTFIT_U16 ? float(static_cast<const uint16_t*>(data)[i])
                              : static_cast<const float*>(data)[i];
}

// Shapes a fit with these limits accepts (the others get NaN start values).
template <int HM>
__device__ __forceinline__ bool usable(const spotfit_shape_t& sh, int max_side, int max_pixels) {
  const int w = sh.w, h = sh.h;
  return !(w < 3 || h < 3 || w > HM || h > HM || w > max_side || h > max_side ||
           w * h > max_pixels || (sh.model != SPOTFIT_SYM && sh.model != SPOTFIT_ELL));
}

__device__ __forceinline__ void write_nan(float* out, int64_t s) {
  const float nanf = __builtin_nanf("");
  for (int q = 0; q < 4; ++q) out[4 * s + q] = nanf;
}

// The k-th smallest of the group's keys (each lane holds RM of them; keys of
// empty slots are all ones): a radix select, two bits per round from the top of
// BITS-bit keys.  Each round counts, over the group, the keys below the three
// candidates prefix|01, prefix|10, prefix|11 (the three counts, at most 124
// each, travel packed in one integer through a single group total) and keeps
// the largest candidate with at most k keys below it.
template <int L, int RM, int BITS>
__device__ __forceinline__ uint32_t select_kth(const uint32_t (&key)[RM], int k) {
  uint32_t v = 0;
#pragma unroll
  for (int shift = BITS - 2; shift >= 0; shift -= 2) {
    const uint32_t c1 = v | (1u << shift), c2 = v | (2u << shift), c3 = v | (3u << shift);
    int cnt = 0;
#pragma unroll
    for (int m = 0; m < RM; ++m)
      cnt += (key[m] < c1 ? 1 : 0) + (key[m] < c2 ? 0x100 : 0) + (key[m] < c3 ? 0x10000 : 0);
    cnt = gsum_i<L>(cnt);
    const uint32_t d = ((cnt & 0xff) <= k ? 1u : 0u) + (((cnt >> 8) & 0xff) <= k ? 1u : 0u) +
                       (((cnt >> 16) & 0xff) <= k ? 1u : 0u);
    v |= d << shift;
  }
  return v;
}

// Background b0: the median of the spot's border ring, on every lane of the group.
template <int L, int CPL>
__device__ __forceinline__ double ring_background(const void* data, int dtype,
                                                  const spotfit_shape_t sh, int64_t off, int li) {
  constexpr int HM = L * CPL;
  constexpr int RM = (4 * HM + L - 1) / L;  // ring pixels per lane, at most
  const int w = sh.w, h = sh.h;
  // keys: the 16-bit values themselves, or order-preserving 32-bit keys of floats
  const bool u16 = dtype == SPOTFIT_U16;
  const int nr = 2 * (w + h - 2);
  uint32_t key[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int qq = li + L * m;
    const int q = qq < nr ? qq : nr - 1;  // slots past the ring re-read its last pixel
    int r = 0, c = 0;
    if (q < w) {
      c = q;
    } else if (q < 2 * w) {
      r = h - 1;
      c = q - w;
    } else if (q < 2 * w + h - 2) {
      r = q - 2 * w + 1;
    } else {
      r = q - 2 * w - (h - 2) + 1;
      c = w - 1;
    }
    const int64_t i = off + r * w + c;
    key[m] = u16 ? uint32_t(static_cast<const uint16_t*>(data)[i])
                 : key_of(static_cast<const float*>(data)[i]);
  }
#pragma unroll
  for (int m = 0; m < RM; ++m) key[m] = li + L * m < nr ? key[m] : 0xFFFFFFFFu;
  const int k1 = nr / 2 - 1;  // the two middle order statistics: k1 and k1 + 1
  const uint32_t v1 = u16 ? select_kth<L, RM, 16>(key, k1) : select_kth<L, RM, 32>(key, k1);
  int le = 0;
  uint32_t above = 0xFFFFFFFFu;
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    le += key[m] <= v1 ? 1 : 0;
    above = (key[m] > v1 && key[m] < above) ? key[m] : above;
  }
  le = gsum_i<L>(le);
  above = gmin_u<L>(above);
  const uint32_t v2 = le >= k1 + 2 ? v1 : above;
  return u16 ? 0.5 * (double(v1) + double(v2))
             : 0.5 * (double(value_of(v1)) + double(value_of(v2)));
}

// Start values o4 from the lane's partial weight moments about the ROI centre
// (sum wt, sum wt dx, sum wt dy, sum wt dx^2, sum wt dy^2): group totals, then
// centroid, variances and the clamped widths.
template <int L>
__device__ __forceinline__ void moment_values(double sw, double swx, double swy, double swxx,
                                              double swyy, const spotfit_shape_t sh, float* o4) {
  const int w = sh.w, h = sh.h;
  const double c0 = 0.5 * (w - 1), r0 = 0.5 * (h - 1);
  sw = gsum<L>(sw);
  swx = gsum<L>(swx);
  swy = gsum<L>(swy);
  swxx = gsum<L>(swxx);
  swyy = gsum<L>(swyy);
  double o[4];
  if (!(sw > 0.0)) {
    o[0] = c0;
    o[1] = r0;
    o[2] = o[3] = 1.5;
  } else {
    const double mx = swx / sw, my = swy / sw;  // centroid relative to the ROI centre
    const double vx = swxx / sw - mx * mx, vy = swyy / sw - my * my;
    double sx, sy;
    if (sh.model == SPOTFIT_SYM) {
      sx = sy = sqrt(0.5 * (vx + vy));
    } else {
      sx = sqrt(vx);
      sy = sqrt(vy);
    }
    const double lo = 0.8, hi = 0.25 * double(w > h ? w : h);
    o[0] = c0 + mx;
    o[1] = r0 + my;
    o[2] = sx < lo ? lo : (sx > hi ? hi : sx);
    o[3] = sy < lo ? lo : (sy > hi ? hi : sy);
  }
  for (int q = 0; q < 4; ++q) o4[q] = float(o[q]);
}

// The start values of one spot, every pixel read from memory: the ring median,
// then the weights' moments in one pass, column by column with the rows streamed.
template <int L, int CPL>
__device__ __forceinline__ void moment_init_spot(const void* data, int dtype, const spotfit_shape_t sh,
                                                 int64_t off, int li, float* o4) {
  const double b0 = ring_background<L, CPL>(data, dtype, sh, off, li);
  const int w = sh.w, h = sh.h;
  const double c0 = 0.5 * (w - 1), r0 = 0.5 * (h - 1);
  double sw = 0.0, swx = 0.0, swy = 0.0, swxx = 0.0, swyy = 0.0;
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = li + L * j;
    if (c >= w) continue;
    const double dx = double(c) - c0;
    double cw = 0.0, cwy = 0.0, cwyy = 0.0;  // this column's sums
#pragma unroll 4
    for (int r = 0; r < h; ++r) {
      const double v = fmax(double(load_px(data, dtype, off + r * w + c)) - b0, 0.0);
      const double dy = double(r) - r0;
      cw += v;
      cwy = __builtin_fma(v, dy, cwy);
      cwyy = __builtin_fma(v * dy, dy, cwyy);
    }
    sw += cw;
    swx = __builtin_fma(cw, dx, swx);
    swxx = __builtin_fma(cw * dx, dx, swxx);
    swy += cwy;
    swyy += cwyy;
  }
  moment_values<L>(sw, swx, swy, swxx, swyy, sh, o4);
}

}  // namespace ini
}  // namespace sf
