// spotfit_track.h -- drift tracking of fiducial markers over the fitted
// positions of a serving loop's frames (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"

namespace sf {

// A tracked frame of one launch: where its markers start in the spot ring and
// its position in the sequence of tracked frames.
struct TrackFrame {
  int64_t spot0;
  int64_t q;
};

// One entry of the device history ring (window entries, indexed q % window).
struct TrackHist {
  double dx, dy;
  int64_t n_used;
};

// Enqueue the drift pass over nf tracked frames (in sequence order) on st.
hipError_t launch_drift_track(const TrackFrame* frames, int nf, const float* params,
                              const int32_t* status, const float* ref_xy, int n_markers,
                              TrackHist* hist, int window, spotfit_drift_t* out, hipStream_t st);

}  // namespace sf
