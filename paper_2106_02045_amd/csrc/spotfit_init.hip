// spotfit_init.hip -- start values on the device: the centroid / second-moment
// estimate from the spot's own pixels.  The paper takes start values as given
// and leaves them out of its timings (Results section); this pass lets raw
// frames go in and fits come out without a host round trip.
//
// Per spot: background b0 = median of the border ring (top row, bottom row,
// then the left and right columns without the corners; the ring has an even
// number of pixels, so b0 is the mean of its two middle values); weights
// wt = max(g - b0, 0); centre = weighted centroid; var_x = sum wt (x - cx)^2 /
// sum wt (var_y alike); symmetric sigma = sqrt((var_x + var_y) / 2), elliptical
// sigma_x = sqrt(var_x), sigma_y = sqrt(var_y); sigmas clamped to
// [0.8, max(w, h) / 4]; with no positive weight: the ROI centre and sigma 1.5.
//
// Mapping: a group of L lanes per spot, lane l owning the columns l + L*j as in
// the fit kernel.  The ring median is a radix select over order-preserving
// 32-bit keys of the ring values (each lane holds every L-th ring pixel; one
// group count per key bit), so no sort and no LDS are needed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lanegroup.h"
#include "spotfit.h"
#include "spotfit_internal.h"

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

template <int L, int CPL>
__global__ __launch_bounds__(64) void moment_init_kernel(const void* data, int dtype,
                                                         const spotfit_shape_t* sizes,
                                                         const int64_t* offsets, int64_t n,
                                                         int max_side, int max_pixels,
                                                         float* out) {
  constexpr int HM = L * CPL;
  constexpr int RM = (4 * HM + L - 1) / L;  // ring pixels per lane, at most
  const int lane = __lane_id();
  const int li = lane % L;
  const int64_t s = (int64_t)blockIdx.x * (64 / L) + lane / L;
  if (s >= n) return;  // whole groups leave together
  const spotfit_shape_t sh = sizes[s];
  const int w = sh.w, h = sh.h;
  if (w < 3 || h < 3 || w > HM || h > HM || w > max_side || h > max_side || w * h > max_pixels ||
      (sh.model != SPOTFIT_SYM && sh.model != SPOTFIT_ELL)) {
    if (li == 0) {
      const float nanf = __builtin_nanf("");
      for (int q = 0; q < 4; ++q) out[4 * s + q] = nanf;
    }
    return;
  }
  const int64_t off = offsets[s];

  // ---- background: median of the border ring ----
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
    key[m] = key_of(load_px(data, dtype, off + r * w + c));
  }
#pragma unroll
  for (int m = 0; m < RM; ++m) key[m] = li + L * m < nr ? key[m] : 0xFFFFFFFFu;
  const int k1 = nr / 2 - 1;  // the two middle order statistics: k1 and k1 + 1
  uint32_t v1 = 0;
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t cand = v1 | (1u << bit);
    int cnt = 0;
#pragma unroll
    for (int m = 0; m < RM; ++m) cnt += key[m] < cand ? 1 : 0;
    if (gsum_i<L>(cnt) <= k1) v1 = cand;
  }
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
  const double b0 = 0.5 * (double(value_of(v1)) + double(value_of(v2)));

  // ---- weights, centroid, second moments ----
  // every slot loaded at once (clamped into the spot), masked afterwards
  float gv[CPL][HM];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = li + L * j < w ? li + L * j : w - 1;
#pragma unroll
    for (int r = 0; r < HM; ++r) gv[j][r] = load_px(data, dtype, off + (r < h ? r : h - 1) * w + c);
  }
  double wt[CPL][HM];
  double sw = 0.0, swx = 0.0, swy = 0.0;
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int c = li + L * j;
#pragma unroll
    for (int r = 0; r < HM; ++r) {
      const double v = (c < w && r < h) ? fmax(double(gv[j][r]) - b0, 0.0) : 0.0;
      wt[j][r] = v;
      sw += v;
      swx = __builtin_fma(v, double(c), swx);
      swy = __builtin_fma(v, double(r), swy);
    }
  }
  sw = gsum<L>(sw);
  swx = gsum<L>(swx);
  swy = gsum<L>(swy);
  double o[4];
  if (!(sw > 0.0)) {
    o[0] = 0.5 * (w - 1);
    o[1] = 0.5 * (h - 1);
    o[2] = o[3] = 1.5;
  } else {
    const double cx = swx / sw, cy = swy / sw;
    double vx = 0.0, vy = 0.0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const double dx = double(li + L * j) - cx;
#pragma unroll
      for (int r = 0; r < HM; ++r) {
        const double dy = double(r) - cy;
        vx = __builtin_fma(wt[j][r] * dx, dx, vx);
        vy = __builtin_fma(wt[j][r] * dy, dy, vy);
      }
    }
    vx = gsum<L>(vx) / sw;
    vy = gsum<L>(vy) / sw;
    double sx, sy;
    if (sh.model == SPOTFIT_SYM) {
      sx = sy = sqrt(0.5 * (vx + vy));
    } else {
      sx = sqrt(vx);
      sy = sqrt(vy);
    }
    const double lo = 0.8, hi = 0.25 * double(w > h ? w : h);
    o[0] = cx;
    o[1] = cy;
    o[2] = sx < lo ? lo : (sx > hi ? hi : sx);
    o[3] = sy < lo ? lo : (sy > hi ? hi : sy);
  }
  if (li == 0)
    for (int q = 0; q < 4; ++q) out[4 * s + q] = float(o[q]);
}

}  // namespace ini

hipError_t launch_moment_init(const void* data, int dtype, const spotfit_shape_t* sizes,
                              const int64_t* offsets, int64_t n, int max_side, int max_pixels,
                              float* out, hipStream_t st) {
  const int cls = max_side <= 8 ? 0 : max_side <= 16 ? 1 : 2;
  const int per_block = cls == 2 ? 4 : 16;
  const int64_t blocks = (n + per_block - 1) / per_block;
  if (cls == 0)
    hipLaunchKernelGGL((ini::moment_init_kernel<4, 2>), dim3((unsigned)blocks), dim3(64), 0, st,
                       data, dtype, sizes, offsets, n, max_side, max_pixels, out);
  else if (cls == 1)
    hipLaunchKernelGGL((ini::moment_init_kernel<4, 4>), dim3((unsigned)blocks), dim3(64), 0, st,
                       data, dtype, sizes, offsets, n, max_side, max_pixels, out);
  else
    hipLaunchKernelGGL((ini::moment_init_kernel<16, 2>), dim3((unsigned)blocks), dim3(64), 0, st,
                       data, dtype, sizes, offsets, n, max_side, max_pixels, out);
  return hipGetLastError();
}

}  // namespace sf
