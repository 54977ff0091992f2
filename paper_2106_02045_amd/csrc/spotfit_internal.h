// spotfit_internal.h -- structures shared by the host side of the library and
// its kernels (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"

namespace sf {

// Options as the kernels read them (host copy of spotfit_options_t, validated).
struct KOpts {
  int max_iter;
  int lambda0_exp10;
  int lambda_max_exp10;
  int max_pixels;
  int max_side;
  int pad_;
  double max_error_per_px;
  double min_delta;
  double min_step_rel;
  double tie_tau;
  double sigma_min;
  double sigma_max_frac;
  // the comparison factors of the loop's decisions, formed once on the host
  // (the same double roundings as on the device): kernel arguments live in
  // scalar registers, whereas loop invariants formed in the kernel take vector
  // registers for the whole fit
  double one_minus_tau;        // 1 - tie_tau
  double one_plus_tau;         // 1 + tie_tau
  double one_minus_min_delta;  // 1 - min_delta
};

// Kernel arguments of one fit launch (all pointers are device memory).
struct KArgs {
  const void* data;
  const spotfit_shape_t* sizes;
  const int64_t* offsets;
  const float* init;
  float* init_out;  // not NULL: start values computed in the fit launch, written here
  float* params_out;
  float* chi2_out;
  int32_t* iters_out;
  int32_t* status_out;
  int32_t* evals_out;
  int32_t* queue;  // spot counter of the narrow kernel's uniform launch (context-owned)
  int64_t n;
  int dtype;
  int pad_;
  KOpts opt;
};

// Pixels per lane of the smallest wave kernel able to hold max_pixels.
int ppl_for_pixels(int max_pixels);
const void* wave_kernel_symbol(int ppl, int precision);
hipError_t launch_wave_kernel(int ppl, int precision, const KArgs& ka, int grid, hipStream_t st);

// One workgroup per spot with `threads` threads (a multiple of 64, >= max_pixels).
hipError_t launch_plain_kernel(const KArgs& ka, int threads, hipStream_t st);

// Device workspace of mixed-size batches: counters[0..2] spots per size class,
// counters[3..5] spots taken; lists: 3 regions of `cap` spot indices.  The
// classify pass orders each class's list by the spots' larger side (a counting
// sort: `sort` holds its per-side counts and cursors), so that the groups of a
// wavefront mostly hold spots of one size and its row loops stop at their
// height; lists built elsewhere may be in any order (sort is then unused).
struct MixedWs {
  int32_t* counters;
  int32_t* lists;
  int64_t cap;
  int32_t* sort = nullptr;
};
// Words of a mixed workspace before its lists: 8 counters, then kSortWords for
// the classify pass's counts (larger side 0..32, and 33 for anything above) and
// cursors.
constexpr int kSortBuckets = 34;
constexpr int kSortWords = 128;
constexpr int64_t kMixedHeadWords = 8 + kSortWords;

// Mixed-size batches: reset + classify + one persistent fit launch.
int mixed_plan_count();
const void* mixed_kernel_symbol(int plan);
hipError_t launch_mixed(int plan, const KArgs& ka, const MixedWs& ws, int grid, hipStream_t st);
// The fit of a mixed-size launch whose workspace already holds the class lists
// and counts (taken counters zero), without the classify pass.
hipError_t launch_mixed_fit(int plan, const KArgs& ka, const MixedWs& ws, int grid, hipStream_t st);

// A fit of spots whose size classes the caller listed (options validated,
// double precision, mixed schedule): ws.counters[0..2] the class sizes,
// ws.counters[3..5] zero, class c's spot indices at ws.lists + c * ws.cap, all
// in device memory.  init_out not NULL: start values computed in the launch
// and written there (init unused), as spotfit_fit_raw.  One launch, no
// classify pass.  Returns SPOTFIT_OK or a negative spotfit_error_t.
int fit_preclassified(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                      const spotfit_shape_t* sizes, const int64_t* offsets, const float* init,
                      float* init_out, int64_t n, const spotfit_options_t& o, const MixedWs& ws,
                      float* params_out, float* chi2_out, int32_t* iters_out, int32_t* status_out,
                      void* stream);

// Plans of the separable kernel: plan p groups `lanes` lanes per spot with `cpl`
// columns per lane and holds spots with w, h <= lanes * cpl.  Plans below
// wide_plan_count() keep a group's state in LDS and share its scalar work over
// the lanes; the narrow plans after them keep it in registers on every lane; two
// one-wave builds of wide plans follow, then the lane-owned plans
// (owned_plan_id(lanes, cpl, own): groups of `lanes` lanes with `cpl` columns per
// lane holding `own` spots; shape (lanes / own) x (cpl * own), so that 64 /
// shape lanes is the spots a wavefront holds).  The lane-owned kernel reads its
// start values: a fit that computes them in its launch runs the narrow
// lanes x cpl plan (plan_for_raw).
int group_plan_count();
int owned_plan_id(int lanes, int cpl, int own);
int plan_for_raw(int plan);
void group_plan_shape(int plan, int* lanes, int* cpl);
const void* group_kernel_symbol(int plan);
hipError_t launch_group_kernel(int plan, const KArgs& ka, int grid, hipStream_t st);
int wide_plan_count();

int narrow_plan_count();
void narrow_plan_shape(int plan, int* lanes, int* cpl);
const void* narrow_kernel_symbol(int plan);
// Resets ka.queue, then fits ka.n < 2^31 spots handed out through that counter.
hipError_t launch_narrow_kernel(int plan, const KArgs& ka, int grid, hipStream_t st);
int narrow_mixed_plan_count();
const void* narrow_mixed_kernel_symbol(int plan);
// the lane-owned kernel (spots up to 16 x 16 pixels): resets ka.queue, then
// fits ka.n < 2^31 spots handed out through that counter; reads ka.init
// lanes per group, columns per lane (spots up to lanes * cpl px), spots per
// group; built: (4, 4, 4), (4, 4, 2), (4, 2, 4), (16, 2, 4), (16, 2, 8)
const void* owned_kernel_symbol(int lanes, int cpl, int own);
hipError_t launch_owned_kernel(int lanes, int cpl, int own, const KArgs& ka, int grid, hipStream_t st);
// the mixed-size plan that gives `plan`'s bits with narrow mappings only (the
// lane-owned plan's all-narrow twin), or `plan` itself
int mixed_plan_narrow(int plan);
// the fit launch of a mixed batch whose spots the classify pass has bucketed
hipError_t launch_narrow_mixed_fit(int plan, const KArgs& ka, const MixedWs& ws, int grid,
                                   hipStream_t st);

// Start values from the pixels for spots with sides up to max_side: float[n][4]
// into out.  kInitMoments: centroid / second moments; kInitPeak: the paper's
// recipe (brightest pixel of the 3 x 3 moving average, sigma = sqrt(M / pi)).
enum { kInitMoments = 0, kInitPeak = 1 };
hipError_t launch_start_values(int method, const void* data, int dtype, const spotfit_shape_t* sizes,
                               const int64_t* offsets, int64_t n, int max_side, int max_pixels,
                               float* out, hipStream_t st);

}  // namespace sf
