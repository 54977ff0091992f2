// spotfit_track.hip -- drift of the sample from fiducial markers: their fitted
// positions averaged over the markers of a frame and over the last frames (the
// paper's use of the fit, tracking markers to stabilise the sample,
// Introduction).  Runs inside the serving loop right after a launch's fit, on
// the same stream, so positions never leave the device before the drift is
// formed.
//
// One workgroup walks the launch's tracked frames in sequence order.  Per
// frame: the markers whose fit stopped on a convergence test (MAX_ERROR,
// MIN_DELTA or MIN_STEP) with finite x and y count; (dx, dy) = mean over them
// of (x - ref_x, y - ref_y), summed in double (threads stride over the markers,
// then a tree in LDS); the entry goes into the history ring; (Dx, Dy) = mean of
// the entries of the last `window` tracked frames that had a counted marker.
// The serving loop chains consecutive launches' passes with an event, so the
// ring is always written in sequence order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "spotfit_track.h"

namespace sf {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void block_sum3(double& a, double& b, int64_t& c, double* sa,
                                           double* sb, int64_t* sc) {
  const int t = threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  sc[t] = c;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      sa[t] += sa[t + h];
      sb[t] += sb[t + h];
      sc[t] += sc[t + h];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  c = sc[0];
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void drift_track_kernel(
    const TrackFrame* frames, int nf, const float* params, const int32_t* status,
    const float* ref_xy, int n_markers, TrackHist* hist, int window, spotfit_drift_t* out) {
  __shared__ double sa[kThreads], sb[kThreads];
  __shared__ int64_t sc[kThreads];
  const int t = threadIdx.x;
  const double nan = __builtin_nan("");
  for (int f = 0; f < nf; ++f) {
    const int64_t s0 = frames[f].spot0, q = frames[f].q;
    double ax = 0.0, ay = 0.0;
    int64_t an = 0;
    for (int k = t; k < n_markers; k += kThreads) {
      const int st = status[s0 + k];
      const float x = params[6 * (s0 + k)], y = params[6 * (s0 + k) + 1];
      if ((st == SPOTFIT_MAX_ERROR || st == SPOTFIT_MIN_DELTA || st == SPOTFIT_MIN_STEP) &&
          __builtin_isfinite(x) && __builtin_isfinite(y)) {
        ax += double(x) - double(ref_xy[2 * k]);
        ay += double(y) - double(ref_xy[2 * k + 1]);
        ++an;
      }
    }
    block_sum3(ax, ay, an, sa, sb, sc);
    const double dx = an > 0 ? ax / double(an) : nan;
    const double dy = an > 0 ? ay / double(an) : nan;
    if (t == 0) hist[q % window] = TrackHist{dx, dy, an};
    __syncthreads();
    const int64_t m = q + 1 < window ? q + 1 : window;
    double bx = 0.0, by = 0.0;
    int64_t bn = 0;
    for (int64_t j = t; j < m; j += kThreads) {
      const TrackHist e = hist[(q - j) % window];
      if (e.n_used > 0) {
        bx += e.dx;
        by += e.dy;
        ++bn;
      }
    }
    block_sum3(bx, by, bn, sa, sb, sc);
    if (t == 0) {
      spotfit_drift_t r;
      r.dx = float(dx);
      r.dy = float(dy);
      r.mean_dx = bn > 0 ? float(bx / double(bn)) : __builtin_nanf("");
      r.mean_dy = bn > 0 ? float(by / double(bn)) : __builtin_nanf("");
      r.n_used = (int32_t)an;
      r.n_frames = (int32_t)bn;
      out[f] = r;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_drift_track(const TrackFrame* frames, int nf, const float* params,
                              const int32_t* status, const float* ref_xy, int n_markers,
                              TrackHist* hist, int window, spotfit_drift_t* out, hipStream_t st) {
  hipLaunchKernelGGL(drift_track_kernel, dim3(1), dim3(kThreads), 0, st, frames, nf, params,
                     status, ref_xy, n_markers, hist, window, out);
  return hipGetLastError();
}

}  // namespace sf
