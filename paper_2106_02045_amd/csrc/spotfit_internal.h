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
};

// Kernel arguments of one fit launch (all pointers are device memory).
struct KArgs {
  const void* data;
  const spotfit_shape_t* sizes;
  const int64_t* offsets;
  const float* init;
  float* params_out;
  float* chi2_out;
  int32_t* iters_out;
  int32_t* status_out;
  int32_t* evals_out;
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

// Lanes per spot of the separable kernel able to hold spots with w, h <= max_side.
int group_lanes_for_side(int max_side);
// wpe: minimum waves per SIMD the register allocation must allow (1..4).
const void* group_kernel_symbol(int lanes, int wpe);
hipError_t launch_group_kernel(int lanes, int wpe, const KArgs& ka, int grid, hipStream_t st);

}  // namespace sf
