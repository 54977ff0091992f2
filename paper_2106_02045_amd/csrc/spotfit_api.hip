// spotfit_api.hip -- host side of the C ABI declared in include/spotfit.h:
// option defaults and validation, the device context and the launch of the fit
// kernels.  Every check runs on the host before any HIP call; the fit itself
// runs entirely on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "spotfit_lm.h"

struct spotfit_ctx {
  int device;
  int n_cu;
  // resident 64-lane workgroups per CU, per (ppl class, per-pixel precision:
  // FP32, MIXED, COMP)
  int occupancy[5][3];
  // separable kernel: plan used for each size class (max side <= 8, <= 16, <= 32)
  // and resident 64-lane workgroups per CU of every plan
  int plan_for_class[3];
  bool plan_forced[3];  // set by the SPOTFIT_GROUP_PLAN override: no switch by batch size
  int occ_plan[16];
  // mixed-size batches: plan and residency of the persistent kernel, workspace
  int mixed_plan;
  bool mixed_forced;  // set by the SPOTFIT_MIXED_PLAN override
  int occ_mixed[8];
  int32_t* ws;      // counters[8] then 3 lists of ws_cap spot indices
  int64_t ws_cap;
  unsigned long long* stats;  // device histogram buffer of spotfit_get_stats
  int32_t* queue;             // spot counter of the narrow kernel's uniform launches
  int32_t* scratch;           // device address of this device's copy of `scratch` (below)
};

// Scratch memory of spotfit_fit_spots_noalloc: word 0 the uniform schedule's
// spot counter; from word 64 (256 bytes in) the mixed schedule's workspace: 8
// counters, the classify pass's 128 words, then its 3 size-class lists of
// SPOTFIT_NOALLOC_MAX_SPOTS spot indices.  Every GPU
// holds its own copy at its own address.  In host code this name only stands
// for the array: kernels get the address that hipGetSymbolAddress returns for
// the current device (kept per device in g_scratch_addr and in each context).
constexpr int64_t kScratchMixedAt = 64;
constexpr int64_t kScratchWords = kScratchMixedAt + sf::kMixedHeadWords + 3 * (int64_t)SPOTFIT_NOALLOC_MAX_SPOTS;
static __device__ __align__(256) int32_t scratch[kScratchWords];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* what) {
  g_last_error = what;
  return code;
}

int fail_hip(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return SPOTFIT_E_HIP;
}

int fail(int code, const std::string& what) { return fail(code, what.c_str()); }
int fail_hip(hipError_t e, const std::string& where) { return fail_hip(e, where.c_str()); }

// Device address of `scratch` on each device, looked up once per device (with
// that device current) by the first context created there.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_addr[kMaxDevices] = {};

// Address of `scratch` on `device`, which must be current.
hipError_t scratch_address(int device, int32_t** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = static_cast<int32_t*>(ptr);
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

int ppl_index(int ppl) {
  switch (ppl) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    case 8: return 3;
    default: return 4;
  }
}

// spotfit_get_stats device buffer: n, status[6], iterations[65], grad, trial
constexpr int kStatsLen = 1 + 6 + 65 + 2;

__global__ void stats_zero_kernel(unsigned long long* buf) {
  if (threadIdx.x < kStatsLen) buf[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void stats_kernel(const int32_t* status, const int32_t* iters,
                                                     const int32_t* evals, int64_t n,
                                                     unsigned long long* buf) {
  __shared__ unsigned int hist[6 + 65];
  __shared__ unsigned long long ev[2];
  for (int i = threadIdx.x; i < 6 + 65; i += blockDim.x) hist[i] = 0u;
  if (threadIdx.x < 2) ev[threadIdx.x] = 0ull;
  __syncthreads();
  unsigned long long gsum = 0, tsum = 0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int st = status[s];
    if (st >= 0 && st < 6) atomicAdd(&hist[st], 1u);
    const int it = iters[s];
    atomicAdd(&hist[6 + (it < 0 ? 0 : it > 64 ? 64 : it)], 1u);
    if (evals) {
      gsum += (unsigned long long)(evals[2 * s] > 0 ? evals[2 * s] : 0);
      tsum += (unsigned long long)(evals[2 * s + 1] > 0 ? evals[2 * s + 1] : 0);
    }
  }
  if (gsum) atomicAdd(&ev[0], gsum);
  if (tsum) atomicAdd(&ev[1], tsum);
  __syncthreads();
  for (int i = threadIdx.x; i < 6 + 65; i += blockDim.x)
    if (hist[i]) atomicAdd(&buf[1 + i], (unsigned long long)hist[i]);
  if (threadIdx.x < 2 && ev[threadIdx.x]) atomicAdd(&buf[1 + 6 + 65 + threadIdx.x], ev[threadIdx.x]);
  if (blockIdx.x == 0 && threadIdx.x == 0) buf[0] = (unsigned long long)n;
}

// y = e^x with the fit kernels' own exponential (grid-stride over n values)
__global__ __launch_bounds__(256) void exp_neg_kernel(const double* x, double* y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = sf::lm::exp_neg(x[i]);
}

}  // namespace

extern "C" {

void spotfit_default_options(spotfit_options_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->max_iter = 20;               // Results section: at most 20 iterations
  o->lambda0_exp10 = -2;          // LM section: initial damping 0.01
  o->lambda_max_exp10 = 4;        // LM section: stop once damping would exceed 1e4
  o->precision = SPOTFIT_PREC_FP64;
  o->max_error_per_px = 1.0 / 3.0;  // Results section: chi^2 < A/3, A = pixel count
  o->min_delta = 1e-6;            // Results section: decrease below 1e-6 chi^2
  o->min_step_rel = 1e-4;         // Results section: |dp_j| < 1e-4 |p_j|
  o->tie_tau = 0.0;
  o->sigma_min = 0.3;
  o->sigma_max_frac = 1.0;
  o->max_pixels = 1024;           // Implementation section: at most 1024 pixels per fit
  o->max_side = 32;
  o->schedule = SPOTFIT_SCHEDULE_UNIFORM;
  o->plan_hint = SPOTFIT_PLAN_THROUGHPUT;
}

int spotfit_validate_options(const spotfit_options_t* o) {
  if (!o) return fail(SPOTFIT_E_NULL, "options: NULL");
  if (o->max_iter < 0 || o->max_iter > 1000) return fail(SPOTFIT_E_OPTIONS, "max_iter not in [0, 1000]");
  if (o->lambda0_exp10 < -300 || o->lambda0_exp10 > 300 || o->lambda_max_exp10 < -300 ||
      o->lambda_max_exp10 > 300)
    return fail(SPOTFIT_E_OPTIONS, "lambda exponents not in [-300, 300]");
  if (o->precision != SPOTFIT_PREC_FP32 && o->precision != SPOTFIT_PREC_MIXED &&
      o->precision != SPOTFIT_PREC_FP64 && o->precision != SPOTFIT_PREC_FP32_PLAIN &&
      o->precision != SPOTFIT_PREC_COMP)
    return fail(SPOTFIT_E_OPTIONS, "unknown precision");
  if (!std::isfinite(o->max_error_per_px) || o->max_error_per_px < 0)
    return fail(SPOTFIT_E_OPTIONS, "max_error_per_px must be finite and >= 0");
  if (!std::isfinite(o->min_delta) || o->min_delta < 0 || o->min_delta >= 1)
    return fail(SPOTFIT_E_OPTIONS, "min_delta not in [0, 1)");
  if (!std::isfinite(o->min_step_rel) || o->min_step_rel < 0)
    return fail(SPOTFIT_E_OPTIONS, "min_step_rel must be finite and >= 0");
  if (!std::isfinite(o->tie_tau) || o->tie_tau < 0 || o->tie_tau >= 1)
    return fail(SPOTFIT_E_OPTIONS, "tie_tau not in [0, 1)");
  if (!std::isfinite(o->sigma_min) || o->sigma_min <= 0)
    return fail(SPOTFIT_E_OPTIONS, "sigma_min must be > 0");
  if (!std::isfinite(o->sigma_max_frac) || o->sigma_max_frac * 3.0 <= o->sigma_min)
    return fail(SPOTFIT_E_OPTIONS, "sigma_max_frac * 3 must exceed sigma_min");
  if (o->max_pixels < 9 || o->max_pixels > 1024)
    return fail(SPOTFIT_E_OPTIONS, "max_pixels not in [9, 1024]");
  if (o->max_side < 3 || o->max_side > 32)
    return fail(SPOTFIT_E_OPTIONS, "max_side not in [3, 32]");
  if (o->schedule != SPOTFIT_SCHEDULE_UNIFORM && o->schedule != SPOTFIT_SCHEDULE_MIXED)
    return fail(SPOTFIT_E_OPTIONS, "unknown schedule");
  if (o->plan_hint != SPOTFIT_PLAN_THROUGHPUT && o->plan_hint != SPOTFIT_PLAN_LATENCY)
    return fail(SPOTFIT_E_OPTIONS, "unknown plan hint");
  return SPOTFIT_OK;
}

int spotfit_ctx_create(spotfit_ctx_t** out, int device) {
  if (!out) return fail(SPOTFIT_E_NULL, "ctx_create: NULL out pointer");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(SPOTFIT_E_DEVICE, "ctx_create: no such device");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SPOTFIT_E_DEVICE, "ctx_create: device is not gfx950");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  spotfit_ctx* c = new (std::nothrow) spotfit_ctx();
  if (!c) return fail(SPOTFIT_E_DEVICE, "ctx_create: out of host memory");
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  const int ppls[5] = {1, 2, 4, 8, 16};
  for (int i = 0; i < 5; ++i) {
    for (int pr = 0; pr < 3; ++pr) {
      const int prec = pr == 0 ? SPOTFIT_PREC_FP32 : pr == 1 ? SPOTFIT_PREC_MIXED : SPOTFIT_PREC_COMP;
      int nb = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sf::wave_kernel_symbol(ppls[i], prec), 64, 0);
      if (e != hipSuccess) {
        delete c;
        return fail_hip(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
      }
      c->occupancy[i][pr] = nb > 0 ? nb : 1;
    }
  }
  for (int pl = 0; pl < sf::group_plan_count(); ++pl) {
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sf::group_kernel_symbol(pl), 64, 0);
    if (e != hipSuccess) {
      delete c;
      return fail_hip(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    }
    c->occ_plan[pl] = nb > 0 ? nb : 1;
  }
  for (int pl = 0; pl < sf::mixed_plan_count(); ++pl) {
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sf::mixed_kernel_symbol(pl), 64, 0);
    if (e != hipSuccess) {
      delete c;
      return fail_hip(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    }
    c->occ_mixed[pl] = nb > 0 ? nb : 1;
  }
  // default mixed-size plan (the last): narrow 4x2 lanes x columns for <= 8 px,
  // lane-owned 4-lane groups of 4 spots for <= 16 px, lane-owned 16-lane groups of
  // 4 spots for <= 32 px
  c->mixed_plan = sf::mixed_plan_count() - 1;
  if (const char* env = std::getenv("SPOTFIT_MIXED_PLAN")) {
    const int v = std::atoi(env);
    if (v >= 0 && v < sf::mixed_plan_count()) {
      c->mixed_plan = v;
      c->mixed_forced = true;
    }
  }
  c->ws = nullptr;
  c->ws_cap = 0;
  c->stats = nullptr;
  c->queue = nullptr;
  c->scratch = nullptr;
  e = scratch_address(device, &c->scratch);
  if (e != hipSuccess) {
    delete c;
    return fail_hip(e, "hipGetSymbolAddress (no-allocation scratch)");
  }
  e = hipMalloc((void**)&c->stats, sizeof(unsigned long long) * kStatsLen);
  if (e == hipSuccess) e = hipMalloc((void**)&c->queue, 256);
  if (e != hipSuccess) {
    if (c->stats) (void)hipFree(c->stats);
    delete c;
    return fail_hip(e, "hipMalloc (context buffers)");
  }
  // default plan per size class (measured on MI355X), all lane-owned (taken for
  // batches large enough, else the narrow plan of the same bits): <= 8 px side:
  // 4-lane groups of 4 spots, 2 columns per lane; <= 16: 4 columns per lane;
  // <= 32: 16-lane groups of 4 spots, 2 columns per lane
  c->plan_for_class[0] = sf::owned_plan_id(4, 2, 4);
  c->plan_for_class[1] = sf::owned_plan_id(4, 4, 4);
  c->plan_for_class[2] = sf::owned_plan_id(16, 2, 4);
  if (const char* env = std::getenv("SPOTFIT_GROUP_PLAN")) {
    // tuning override "a,b,c": plan for each size class
    int a = -1, b = -1, d = -1;
    if (std::sscanf(env, "%d,%d,%d", &a, &b, &d) == 3) {
      const int want[3] = {a, b, d};
      const int side[3] = {8, 16, 32};
      for (int i = 0; i < 3; ++i) {
        int L = 0, C = 0;
        sf::group_plan_shape(want[i], &L, &C);
        if (L * C >= side[i]) {
          c->plan_for_class[i] = want[i];
          c->plan_forced[i] = true;
        }
      }
    }
  }
  if (const char* env = std::getenv("SPOTFIT_WAVES_PER_CU")) {
    const int v = std::atoi(env);
    if (v > 0 && v <= 64) {
      for (int i = 0; i < 5; ++i) c->occupancy[i][0] = c->occupancy[i][1] = c->occupancy[i][2] = v;
      for (int i = 0; i < 16; ++i) c->occ_plan[i] = v;
    }
  }
  *out = c;
  return SPOTFIT_OK;
}

void spotfit_ctx_destroy(spotfit_ctx_t* ctx) {
  if (!ctx) return;
  if (ctx->ws || ctx->stats || ctx->queue) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ctx->device);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->stats) (void)hipFree(ctx->stats);
    if (ctx->queue) (void)hipFree(ctx->queue);
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  delete ctx;
}

int spotfit_ctx_reserve(spotfit_ctx_t* ctx, int64_t n) {
  if (!ctx) return fail(SPOTFIT_E_NULL, "ctx_reserve: NULL context");
  if (n < 0 || n > ((int64_t)1 << 31) - 1) return fail(SPOTFIT_E_ARG, "ctx_reserve: n not in [0, 2^31)");
  if (n <= ctx->ws_cap) return SPOTFIT_OK;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (cur != ctx->device && (e = hipSetDevice(ctx->device)) != hipSuccess)
    return fail_hip(e, "hipSetDevice");
  if (ctx->ws) {
    e = hipDeviceSynchronize();  // a previous call may still use the old workspace
    if (e == hipSuccess) e = hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
  }
  int32_t* p = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&p, sizeof(int32_t) * (size_t)(sf::kMixedHeadWords + 3 * n));
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc (mixed workspace)");
  ctx->ws = p;
  ctx->ws_cap = n;
  return SPOTFIT_OK;
}

}  // extern "C"

namespace {

// Checks of a fit call that need no HIP call; fills the validated options.
int check_call(spotfit_ctx_t* ctx, const void* data, int32_t dtype, const spotfit_shape_t* sizes,
               const int64_t* offsets, const float* init, int64_t n, const spotfit_options_t* opt,
               float* params_out, float* chi2_out, int32_t* iters_out, int32_t* status_out,
               spotfit_options_t* o, const char* who, bool init_optional = false) {
  if (!ctx) return fail(SPOTFIT_E_NULL, (std::string(who) + ": NULL context").c_str());
  if (n < 0) return fail(SPOTFIT_E_ARG, (std::string(who) + ": n_spots < 0").c_str());
  if (dtype != SPOTFIT_U16 && dtype != SPOTFIT_F32)
    return fail(SPOTFIT_E_ARG, (std::string(who) + ": unknown dtype").c_str());
  if (opt) {
    *o = *opt;
  } else {
    spotfit_default_options(o);
  }
  int rc = spotfit_validate_options(o);
  if (rc != SPOTFIT_OK) return rc;
  if (n == 0) return SPOTFIT_OK;
  if (!data || !sizes || !offsets || (!init && !init_optional) || !params_out || !chi2_out ||
      !iters_out || !status_out)
    return fail(SPOTFIT_E_NULL, (std::string(who) + ": NULL array").c_str());
  return SPOTFIT_OK;
}

// Largest batch for which the latency hint takes the one-wave-per-SIMD build
// of the wide mixed-size plan (measured: faster up to 40,000 spots of the
// serving and mixed workloads, slower from 400,000).
constexpr int64_t kLeanMaxSpots = 65536;
// The lane-owned plans hold 16-64 spots per wavefront and make a pass per
// spot of a group each step: they pay off when every resident spot slot fits
// several spots in turn; a smaller batch takes the narrow plan of the same
// bits.  Spots per resident slot from which a uniform launch takes the
// lane-owned plan, in halves: the crossovers measured against the narrow
// plans (15x15: between 262k and 393k spots, 2.0-3.0 per slot; 7x7: between
// 131k and 197k, 1.0-1.5; 32x32: between 66k and 131k, 2.0-4.0); plans that
// are not defaults keep 4.
int64_t owned_min_halves(int plan) {
  if (plan == sf::owned_plan_id(4, 4, 4) || plan == sf::owned_plan_id(16, 2, 4)) return 5;
  if (plan == sf::owned_plan_id(4, 2, 4)) return 3;
  return 8;
}
// The same rule for a mixed-size launch with lane-owned classes (over the
// whole batch; measured at 2M spots only).
constexpr int64_t kOwnedMinSpotsPerLane = 4;

// Enqueue one fit with validated options o and n > 0.  init_out not NULL (with
// init NULL): the separable double-precision kernels compute the start values
// themselves and write them there.  Mixed schedule: `classified` is a
// workspace whose class lists are already built (no classify pass); otherwise
// `own_ws` (not NULL: a workspace of at least n spots that the caller owns) or
// the context's workspace, grown to n spots if needed, takes the classify pass.
int launch_fit(spotfit_ctx_t* ctx, const void* data, int32_t dtype, const spotfit_shape_t* sizes,
               const int64_t* offsets, const float* init, int64_t n, const spotfit_options_t& o,
               float* params_out, float* chi2_out, int32_t* iters_out, int32_t* status_out,
               int32_t* evals_out, void* stream, float* init_out = nullptr,
               const sf::MixedWs* classified = nullptr, const sf::MixedWs* own_ws = nullptr,
               int32_t* own_queue = nullptr) {
  sf::KArgs ka;
  std::memset(&ka, 0, sizeof ka);
  ka.data = data;
  ka.sizes = sizes;
  ka.offsets = offsets;
  ka.init = init;
  ka.init_out = init_out;
  ka.params_out = params_out;
  ka.chi2_out = chi2_out;
  ka.iters_out = iters_out;
  ka.status_out = status_out;
  ka.evals_out = evals_out;
  ka.queue = own_queue ? own_queue : ctx->queue;
  ka.n = n;
  ka.dtype = dtype;
  ka.opt.max_iter = o.max_iter;
  ka.opt.lambda0_exp10 = o.lambda0_exp10;
  ka.opt.lambda_max_exp10 = o.lambda_max_exp10;
  ka.opt.max_pixels = o.max_pixels;
  ka.opt.max_side = o.max_side;
  ka.opt.max_error_per_px = o.max_error_per_px;
  ka.opt.min_delta = o.min_delta;
  ka.opt.min_step_rel = o.min_step_rel;
  ka.opt.tie_tau = o.tie_tau;
  ka.opt.one_minus_tau = 1.0 - o.tie_tau;
  ka.opt.one_plus_tau = 1.0 + o.tie_tau;
  ka.opt.one_minus_min_delta = 1.0 - o.min_delta;
  ka.opt.sigma_min = o.sigma_min;
  ka.opt.sigma_max_frac = o.sigma_max_frac;

  hipError_t e;
  if (o.precision == SPOTFIT_PREC_FP64 && o.schedule == SPOTFIT_SCHEDULE_MIXED) {
    if (!classified && !own_ws && n > ctx->ws_cap) {
      const int rr = spotfit_ctx_reserve(ctx, n);
      if (rr != SPOTFIT_OK) return rr;
    }
    const sf::MixedWs ws = classified ? *classified
                           : own_ws   ? *own_ws
                                      : sf::MixedWs{ctx->ws, ctx->ws + sf::kMixedHeadWords, ctx->ws_cap,
                                                    ctx->ws + 8};
    // latency: the wide mixed-size plan (8, 16, 32 lanes per spot); up to
    // kLeanMaxSpots spots its one-wave-per-SIMD build, which spills no
    // registers (those batches leave most of the chip idle anyway)
    int mplan = o.plan_hint == SPOTFIT_PLAN_LATENCY ? (n <= kLeanMaxSpots ? 3 : 0)
                                                    : ctx->mixed_plan;
    if (sf::mixed_plan_narrow(mplan) != mplan && !ctx->mixed_forced &&
        n < kOwnedMinSpotsPerLane * (int64_t)ctx->n_cu * ctx->occ_mixed[mplan] * 64)
      mplan = sf::mixed_plan_narrow(mplan);
    const int64_t resident = (int64_t)ctx->n_cu * ctx->occ_mixed[mplan];
    const int64_t need = (n + 1) / 2;
    const int grid = (int)(need < resident ? need : resident);
    e = classified ? sf::launch_mixed_fit(mplan, ka, ws, grid, (hipStream_t)stream)
                   : sf::launch_mixed(mplan, ka, ws, grid, (hipStream_t)stream);
  } else if (o.precision == SPOTFIT_PREC_FP64) {
    const int cls = o.max_side <= 8 ? 0 : o.max_side <= 16 ? 1 : 2;
    // latency: the wide plans with one lane per column (8x1, 16x1, 32x1); the
    // builds of 16x1 and 32x1 that spill no registers for batches that they hold
    // resident at once (measured: up to 5-10 % faster there, 10-35 % slower at
    // several resident rounds)
    const int one_wave = sf::wide_plan_count() + sf::narrow_plan_count();
    const int wide_for_class[3] = {0, 2, 4}, lean_for_class[3] = {0, one_wave, one_wave + 1};
    int plan = ctx->plan_for_class[cls];
    if (sf::plan_for_raw(plan) != plan) {  // a lane-owned plan
      int ol = 0, oc = 0;
      sf::group_plan_shape(plan, &ol, &oc);
      const int64_t lanes_resident = (int64_t)ctx->n_cu * ctx->occ_plan[plan] * (64 / ol);
      if (init_out || (!ctx->plan_forced[cls] && 2 * n < owned_min_halves(plan) * lanes_resident))
        plan = sf::plan_for_raw(plan);
    }
    int lanes = 0, cpl = 0;
    if (o.plan_hint == SPOTFIT_PLAN_LATENCY) {
      plan = wide_for_class[cls];
      const int lean = lean_for_class[cls];
      sf::group_plan_shape(lean, &lanes, &cpl);
      if (lean != plan && n <= (int64_t)ctx->n_cu * ctx->occ_plan[lean] * (64 / lanes)) plan = lean;
    }
    sf::group_plan_shape(plan, &lanes, &cpl);
    const int64_t per_wave = 64 / lanes;
    const int64_t need = (n + per_wave - 1) / per_wave;
    // persistent grid: as many one-wave workgroups as can be resident at once
    const int64_t resident = (int64_t)ctx->n_cu * ctx->occ_plan[plan];
    const int grid = (int)(need < resident ? need : resident);
    // the narrow kernel's spot counter is 32-bit: batches of up to 2^30 spots per launch
    const int64_t chunk = (int64_t)1 << 30;
    e = hipSuccess;
    for (int64_t c0 = 0; c0 < n && e == hipSuccess; c0 += chunk) {
      sf::KArgs kc = ka;
      kc.n = n - c0 < chunk ? n - c0 : chunk;
      kc.sizes = sizes + c0;
      kc.offsets = offsets + c0;
      kc.init = init ? init + 4 * c0 : nullptr;
      kc.init_out = init_out ? init_out + 4 * c0 : nullptr;
      kc.params_out = params_out + 6 * c0;
      kc.chi2_out = chi2_out + c0;
      kc.iters_out = iters_out + c0;
      kc.status_out = status_out + c0;
      kc.evals_out = evals_out ? evals_out + 2 * c0 : nullptr;
      e = sf::launch_group_kernel(plan, kc, grid, (hipStream_t)stream);
    }
  } else if (o.precision == SPOTFIT_PREC_FP32_PLAIN) {
    const int threads = ((o.max_pixels + 63) / 64) * 64;
    e = sf::launch_plain_kernel(ka, threads, (hipStream_t)stream);
  } else {
    const int ppl = sf::ppl_for_pixels(o.max_pixels);
    const int pr = o.precision == SPOTFIT_PREC_MIXED ? 1 : o.precision == SPOTFIT_PREC_COMP ? 2 : 0;
    const int64_t resident = (int64_t)ctx->n_cu * ctx->occupancy[ppl_index(ppl)][pr];
    const int grid = (int)(n < resident ? n : resident);
    e = sf::launch_wave_kernel(ppl, o.precision, ka, grid, (hipStream_t)stream);
  }
  if (e != hipSuccess) return fail_hip(e, "fit kernel launch");
  return SPOTFIT_OK;
}

// Whether a fit of n spots with start values in memory (validated options o)
// takes a lane-owned plan: the plan choice of launch_fit.
bool takes_owned(const spotfit_ctx_t* ctx, int64_t n, const spotfit_options_t& o) {
  if (o.precision != SPOTFIT_PREC_FP64 || o.plan_hint == SPOTFIT_PLAN_LATENCY) return false;
  if (o.schedule == SPOTFIT_SCHEDULE_MIXED) {
    const int mplan = ctx->mixed_plan;
    return sf::mixed_plan_narrow(mplan) != mplan &&
           (ctx->mixed_forced || n >= kOwnedMinSpotsPerLane * (int64_t)ctx->n_cu * ctx->occ_mixed[mplan] * 64);
  }
  const int cls = o.max_side <= 8 ? 0 : o.max_side <= 16 ? 1 : 2;
  const int plan = ctx->plan_for_class[cls];
  if (sf::plan_for_raw(plan) == plan) return false;
  int ol = 0, oc = 0;
  sf::group_plan_shape(plan, &ol, &oc);
  const int64_t lanes_resident = (int64_t)ctx->n_cu * ctx->occ_plan[plan] * (64 / ol);
  return ctx->plan_forced[cls] || 2 * n >= owned_min_halves(plan) * lanes_resident;
}

// Enqueue start values and fit (validated options o, n > 0).  The separable
// double-precision kernels of the narrow and wide plans compute them in the
// fit's own launch; a batch that takes a lane-owned plan, and the other
// kernels, get a start-value launch first and read them from memory (the
// lane-owned fit with its start values from memory is the faster of the two
// there: 1M 15x15 1.54 against 1.61 ms, 1M 32x32 5.14 against 6.14, 2M mixed
// sizes 6.45 against 7.11; the same bits either way).
int launch_raw(spotfit_ctx_t* ctx, const void* data, int32_t dtype, const spotfit_shape_t* sizes,
               const int64_t* offsets, int64_t n, const spotfit_options_t& o, float* init_out,
               float* params_out, float* chi2_out, int32_t* iters_out, int32_t* status_out,
               int32_t* evals_out, void* stream, const sf::MixedWs* own_ws = nullptr) {
  if (o.precision == SPOTFIT_PREC_FP64 && !takes_owned(ctx, n, o))
    return launch_fit(ctx, data, dtype, sizes, offsets, nullptr, n, o, params_out, chi2_out,
                      iters_out, status_out, evals_out, stream, init_out, nullptr, own_ws);
  const hipError_t e = sf::launch_start_values(sf::kInitMoments, data, dtype, sizes, offsets, n,
                                               o.max_side, o.max_pixels, init_out,
                                               (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "start-value kernel launch");
  return launch_fit(ctx, data, dtype, sizes, offsets, init_out, n, o, params_out, chi2_out,
                    iters_out, status_out, evals_out, stream, nullptr, nullptr, own_ws);
}

}  // namespace

namespace sf {

int fit_preclassified(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                      const spotfit_shape_t* sizes, const int64_t* offsets, const float* init,
                      float* init_out, int64_t n, const spotfit_options_t& o, const MixedWs& ws,
                      float* params_out, float* chi2_out, int32_t* iters_out, int32_t* status_out,
                      void* stream) {
  if (o.precision != SPOTFIT_PREC_FP64 || o.schedule != SPOTFIT_SCHEDULE_MIXED)
    return fail(SPOTFIT_E_OPTIONS, "fit_preclassified: double precision, mixed schedule only");
  if (n == 0) return SPOTFIT_OK;
  return launch_fit(ctx, data, dtype, sizes, offsets, init_out ? nullptr : init, n, o, params_out,
                    chi2_out, iters_out, status_out, nullptr, stream, init_out, &ws);
}

}  // namespace sf

extern "C" {

int spotfit_fit_spots(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                      const spotfit_shape_t* sizes, const int64_t* offsets, const float* init,
                      int64_t n, const spotfit_options_t* opt, float* params_out,
                      float* chi2_out, int32_t* iters_out, int32_t* status_out,
                      int32_t* evals_out, void* stream) {
  spotfit_options_t o;
  int rc = check_call(ctx, data, dtype, sizes, offsets, init, n, opt, params_out, chi2_out,
                      iters_out, status_out, &o, "fit_spots");
  if (rc != SPOTFIT_OK || n == 0) return rc;
  return launch_fit(ctx, data, dtype, sizes, offsets, init, n, o, params_out, chi2_out, iters_out,
                    status_out, evals_out, stream);
}

int spotfit_fit_spots_noalloc(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                              const spotfit_shape_t* sizes, const int64_t* offsets,
                              const float* init, int64_t n, const spotfit_options_t* opt,
                              float* params_out, float* chi2_out, int32_t* iters_out,
                              int32_t* status_out, int32_t* evals_out, void* stream) {
  spotfit_options_t o;
  int rc = check_call(ctx, data, dtype, sizes, offsets, init, n, opt, params_out, chi2_out,
                      iters_out, status_out, &o, "fit_spots_noalloc");
  if (rc != SPOTFIT_OK || n == 0) return rc;
  if (o.precision == SPOTFIT_PREC_FP64 && o.schedule == SPOTFIT_SCHEDULE_MIXED &&
      n > (int64_t)SPOTFIT_NOALLOC_MAX_SPOTS)
    return fail(SPOTFIT_E_ARG, "fit_spots_noalloc: a mixed-schedule call takes at most "
                               "SPOTFIT_NOALLOC_MAX_SPOTS (1048576) spots");
  if (!ctx->scratch) return fail(SPOTFIT_E_DEVICE, "fit_spots_noalloc: no scratch address");
  // the counters and lists live in this device's copy of `scratch`; the
  // kernels that use them clear the counters first (no memset, no allocation)
  const sf::MixedWs ws{ctx->scratch + kScratchMixedAt,
                       ctx->scratch + kScratchMixedAt + sf::kMixedHeadWords,
                       (int64_t)SPOTFIT_NOALLOC_MAX_SPOTS, ctx->scratch + kScratchMixedAt + 8};
  return launch_fit(ctx, data, dtype, sizes, offsets, init, n, o, params_out, chi2_out, iters_out,
                    status_out, evals_out, stream, nullptr, nullptr, &ws, ctx->scratch);
}

int spotfit_fit_raw(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                    const spotfit_shape_t* sizes, const int64_t* offsets, int64_t n,
                    const spotfit_options_t* opt, float* init_out, float* params_out,
                    float* chi2_out, int32_t* iters_out, int32_t* status_out,
                    int32_t* evals_out, void* stream) {
  spotfit_options_t o;
  int rc = check_call(ctx, data, dtype, sizes, offsets, init_out, n, opt, params_out, chi2_out,
                      iters_out, status_out, &o, "fit_raw");
  if (rc != SPOTFIT_OK || n == 0) return rc;
  return launch_raw(ctx, data, dtype, sizes, offsets, n, o, init_out, params_out, chi2_out,
                    iters_out, status_out, evals_out, stream);
}

static int start_values(int method, const char* what, const void* data, int32_t dtype,
                        const spotfit_shape_t* sizes, const int64_t* offsets, int64_t n,
                        const spotfit_options_t* opt, float* init_out, void* stream) {
  if (n < 0) return fail(SPOTFIT_E_ARG, std::string(what) + ": n_spots < 0");
  if (dtype != SPOTFIT_U16 && dtype != SPOTFIT_F32)
    return fail(SPOTFIT_E_ARG, std::string(what) + ": unknown dtype");
  spotfit_options_t o;
  if (opt) {
    o = *opt;
  } else {
    spotfit_default_options(&o);
  }
  const int rc = spotfit_validate_options(&o);
  if (rc != SPOTFIT_OK) return rc;
  if (n == 0) return SPOTFIT_OK;
  if (!data || !sizes || !offsets || !init_out)
    return fail(SPOTFIT_E_NULL, std::string(what) + ": NULL array");
  const hipError_t e = sf::launch_start_values(method, data, dtype, sizes, offsets, n, o.max_side,
                                               o.max_pixels, init_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, std::string(what) + " kernel launch");
  return SPOTFIT_OK;
}

int spotfit_moment_init(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                        const spotfit_shape_t* sizes, const int64_t* offsets, int64_t n,
                        const spotfit_options_t* opt, float* init_out, void* stream) {
  if (!ctx) return fail(SPOTFIT_E_NULL, "moment_init: NULL context");
  return start_values(sf::kInitMoments, "moment_init", data, dtype, sizes, offsets, n, opt,
                      init_out, stream);
}

int spotfit_peak_init(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                      const spotfit_shape_t* sizes, const int64_t* offsets, int64_t n,
                      const spotfit_options_t* opt, float* init_out, void* stream) {
  if (!ctx) return fail(SPOTFIT_E_NULL, "peak_init: NULL context");
  return start_values(sf::kInitPeak, "peak_init", data, dtype, sizes, offsets, n, opt, init_out,
                      stream);
}

int spotfit_get_stats(spotfit_ctx_t* ctx, const int32_t* status, const int32_t* iters,
                      const int32_t* evals, int64_t n, spotfit_stats_t* out, void* stream) {
  if (!ctx || !out) return fail(SPOTFIT_E_NULL, "get_stats: NULL context or output");
  if (n < 0) return fail(SPOTFIT_E_ARG, "get_stats: n_spots < 0");
  std::memset(out, 0, sizeof *out);
  if (n == 0) return SPOTFIT_OK;
  if (!status || !iters) return fail(SPOTFIT_E_NULL, "get_stats: NULL array");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(stats_zero_kernel, dim3(1), dim3(128), 0, st, ctx->stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e, "statistics kernel launch");
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(stats_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, st,
                     status, iters, evals, n, ctx->stats);
  e = hipGetLastError();
  if (e != hipSuccess) return fail_hip(e, "statistics kernel launch");
  unsigned long long h[kStatsLen];
  e = hipMemcpyAsync(h, ctx->stats, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail_hip(e, "statistics copy");
  out->n_spots = (int64_t)h[0];
  for (int i = 0; i < 6; ++i) out->status_count[i] = (int64_t)h[1 + i];
  for (int i = 0; i < 65; ++i) out->iters_hist[i] = (int64_t)h[7 + i];
  out->grad_evals = (int64_t)h[72];
  out->trial_evals = (int64_t)h[73];
  return SPOTFIT_OK;
}

int spotfit_autotune(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                     const spotfit_shape_t* sizes, const int64_t* offsets, const float* init,
                     int64_t n, const spotfit_options_t* opt, float* params_out, float* chi2_out,
                     int32_t* iters_out, int32_t* status_out, int32_t reps,
                     spotfit_tune_report_t* report, void* stream) {
  spotfit_options_t o;
  int rc = check_call(ctx, data, dtype, sizes, offsets, init, n, opt, params_out, chi2_out,
                      iters_out, status_out, &o, "autotune");
  if (rc != SPOTFIT_OK) return rc;
  if (o.precision != SPOTFIT_PREC_FP64)
    return fail(SPOTFIT_E_OPTIONS, "autotune: only the double-precision separable kernel has plans");
  if (reps < 1) return fail(SPOTFIT_E_ARG, "autotune: reps < 1");
  if (n == 0) return fail(SPOTFIT_E_ARG, "autotune: empty batch");
  const bool mixed = o.schedule == SPOTFIT_SCHEDULE_MIXED;
  const int cls = o.max_side <= 8 ? 0 : o.max_side <= 16 ? 1 : 2;
  const int side = cls == 0 ? 8 : cls == 1 ? 16 : 32;
  int cand[16];
  int nc = 0;
  if (mixed) {
    for (int p = 0; p < sf::mixed_plan_count() && nc < 16; ++p) cand[nc++] = p;
  } else {
    for (int p = 0; p < sf::group_plan_count() && nc < 16; ++p) {
      int L = 0, C = 0;
      sf::group_plan_shape(p, &L, &C);
      if (L * C >= side) cand[nc++] = p;
    }
  }
  double ms[16];
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return fail_hip(e, "hipEventCreate");
  const int keep = mixed ? ctx->mixed_plan : ctx->plan_for_class[cls];
  int best = 0;
  for (int i = 0; i < nc && rc == SPOTFIT_OK; ++i) {
    if (mixed)
      ctx->mixed_plan = cand[i];
    else
      ctx->plan_for_class[cls] = cand[i];
    rc = launch_fit(ctx, data, dtype, sizes, offsets, init, n, o, params_out, chi2_out, iters_out,
                    status_out, nullptr, stream);
    if (rc == SPOTFIT_OK && (e = hipEventRecord(e0, st)) != hipSuccess) rc = fail_hip(e, "hipEventRecord");
    for (int r = 0; r < reps && rc == SPOTFIT_OK; ++r)
      rc = launch_fit(ctx, data, dtype, sizes, offsets, init, n, o, params_out, chi2_out,
                      iters_out, status_out, nullptr, stream);
    if (rc == SPOTFIT_OK && (e = hipEventRecord(e1, st)) != hipSuccess) rc = fail_hip(e, "hipEventRecord");
    if (rc == SPOTFIT_OK && (e = hipEventSynchronize(e1)) != hipSuccess) rc = fail_hip(e, "hipEventSynchronize");
    float t = 0.f;
    if (rc == SPOTFIT_OK && (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess)
      rc = fail_hip(e, "hipEventElapsedTime");
    ms[i] = double(t) / reps;
    if (rc == SPOTFIT_OK && ms[i] < ms[best]) best = i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int chosen = rc == SPOTFIT_OK ? cand[best] : keep;
  if (mixed)
    ctx->mixed_plan = chosen;
  else
    ctx->plan_for_class[cls] = chosen;
  if (rc != SPOTFIT_OK) return rc;
  // the outputs: the kept plan's results
  rc = launch_fit(ctx, data, dtype, sizes, offsets, init, n, o, params_out, chi2_out, iters_out,
                  status_out, nullptr, stream);
  if (rc != SPOTFIT_OK) return rc;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  if (report) {
    std::memset(report, 0, sizeof *report);
    report->schedule = o.schedule;
    report->size_class = mixed ? -1 : cls;
    report->n_candidates = nc;
    report->chosen = best;
    for (int i = 0; i < nc; ++i) {
      report->plan_id[i] = cand[i];
      report->plan_ms[i] = ms[i];
    }
  }
  return SPOTFIT_OK;
}

const char* spotfit_last_error(void) { return g_last_error.c_str(); }

int spotfit_version(void) { return 100; }

int spotfit_exp_neg(const double* x, double* y, int64_t n, void* stream) {
  if (n < 0) return fail(SPOTFIT_E_ARG, "exp_neg: n < 0");
  if (n == 0) return SPOTFIT_OK;
  if (!x || !y) return fail(SPOTFIT_E_NULL, "exp_neg: NULL array");
  const int64_t blocks = (n + 255) / 256;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(exp_neg_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, x, y, n);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOTFIT_OK : fail_hip(e, "exp_neg launch");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Captured fits of fixed-shape batches: the copies and kernels of one call,
// recorded once into a HIP graph on a private stream and replayed with one
// launch.
// ---------------------------------------------------------------------------
struct spotfit_graph {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  float* init_buf = nullptr;  // start values of a graph that computes them (init NULL)
  int32_t* ws = nullptr;      // the mixed schedule's workspace, owned by the graph (its
                              // kernels keep this address for every replay)
};

extern "C" {

int spotfit_graph_create(spotfit_graph_t** out, spotfit_ctx_t* ctx, const void* data,
                         int32_t dtype, const spotfit_shape_t* sizes, const int64_t* offsets,
                         const float* init, int64_t n, const spotfit_options_t* opt,
                         float* params_out, float* chi2_out, int32_t* iters_out,
                         int32_t* status_out, const spotfit_graph_io_t* io) {
  if (!out) return fail(SPOTFIT_E_NULL, "graph_create: NULL out pointer");
  *out = nullptr;
  spotfit_options_t o;
  int rc = check_call(ctx, data, dtype, sizes, offsets, init, n, opt, params_out, chi2_out,
                      iters_out, status_out, &o, "graph_create", true);
  if (rc != SPOTFIT_OK) return rc;
  if (n == 0) return fail(SPOTFIT_E_ARG, "graph_create: n_spots = 0");
  const bool raw = init == nullptr;  // start values computed on the device
  if (raw && io && io->init)
    return fail(SPOTFIT_E_ARG, "graph_create: io->init needs a device init array");
  if (io && io->data && io->data_bytes <= 0)
    return fail(SPOTFIT_E_ARG, "graph_create: io->data_bytes must be > 0 with io->data");
  // the caller's current device is restored on return
  struct DeviceGuard {
    int prev = -1;
    ~DeviceGuard() {
      if (prev >= 0) (void)hipSetDevice(prev);
    }
  } guard;
  hipError_t e = hipGetDevice(&guard.prev);
  if (e == hipSuccess) e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
  spotfit_graph* g = new (std::nothrow) spotfit_graph();
  if (!g) return fail(SPOTFIT_E_ARG, "graph_create: out of host memory");
  g->device = ctx->device;
  // the mixed schedule's workspace belongs to the graph and is allocated before the
  // capture: nothing allocates inside it, and a later call that grows the
  // context's workspace cannot free memory the replays use
  const bool mixed = o.precision == SPOTFIT_PREC_FP64 && o.schedule == SPOTFIT_SCHEDULE_MIXED;
  sf::MixedWs gws{nullptr, nullptr, 0};
  if (mixed) {
    e = hipMalloc((void**)&g->ws, sizeof(int32_t) * (size_t)(sf::kMixedHeadWords + 3 * n));
    if (e != hipSuccess) {
      g->ws = nullptr;
      spotfit_graph_destroy(g);
      return fail_hip(e, "hipMalloc (graph workspace)");
    }
    gws = sf::MixedWs{g->ws, g->ws + sf::kMixedHeadWords, n, g->ws + 8};
  }
  if (raw) {
    e = hipMalloc((void**)&g->init_buf, sizeof(float) * 4 * (size_t)n);
    if (e != hipSuccess) {
      g->init_buf = nullptr;
      spotfit_graph_destroy(g);
      return fail_hip(e, "hipMalloc (graph start values)");
    }
  }
  hipStream_t st = nullptr;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    spotfit_graph_destroy(g);
    return fail_hip(e, "hipStreamCreateWithFlags");
  }
  e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess && io && io->data)
    e = hipMemcpyAsync(const_cast<void*>(data), io->data, (size_t)io->data_bytes,
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && io && io->init)
    e = hipMemcpyAsync(const_cast<float*>(init), io->init, sizeof(float) * 4 * (size_t)n,
                       hipMemcpyHostToDevice, st);
  rc = SPOTFIT_OK;
  if (e == hipSuccess && raw)
    rc = launch_raw(ctx, data, dtype, sizes, offsets, n, o, g->init_buf, params_out, chi2_out,
                    iters_out, status_out, nullptr, st, mixed ? &gws : nullptr);
  else if (e == hipSuccess)
    rc = launch_fit(ctx, data, dtype, sizes, offsets, init, n, o, params_out, chi2_out, iters_out,
                    status_out, nullptr, st, nullptr, nullptr, mixed ? &gws : nullptr);
  if (e == hipSuccess && rc == SPOTFIT_OK && io && io->params)
    e = hipMemcpyAsync(io->params, params_out, sizeof(float) * 6 * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && rc == SPOTFIT_OK && io && io->chi2)
    e = hipMemcpyAsync(io->chi2, chi2_out, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && rc == SPOTFIT_OK && io && io->iters)
    e = hipMemcpyAsync(io->iters, iters_out, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && rc == SPOTFIT_OK && io && io->status)
    e = hipMemcpyAsync(io->status, status_out, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st);
  // always end the capture, so the stream leaves capture mode whatever failed
  const hipError_t e_end = hipStreamEndCapture(st, &g->graph);
  if (e == hipSuccess) e = e_end;
  if (e == hipSuccess && rc == SPOTFIT_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(st);
  if (e != hipSuccess || rc != SPOTFIT_OK) {
    const std::string why = rc != SPOTFIT_OK ? std::string(spotfit_last_error()) : hipGetErrorString(e);
    spotfit_graph_destroy(g);
    return rc != SPOTFIT_OK ? fail(rc, "graph_create: " + why) : fail_hip(e, "graph_create");
  }
  *out = g;
  return SPOTFIT_OK;
}

int spotfit_graph_launch(spotfit_graph_t* g, void* stream) {
  if (!g || !g->exec) return fail(SPOTFIT_E_NULL, "graph_launch: NULL graph");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
  return SPOTFIT_OK;
}

void spotfit_graph_destroy(spotfit_graph_t* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->init_buf) (void)hipFree(g->init_buf);
  if (g->ws) (void)hipFree(g->ws);
  delete g;
}

}  // extern "C"
