/*
 * spotfit.h -- C ABI of the MI355X (gfx950) batched Gaussian-spot fitter.
 *
 * Fits many small image spots (at most 1024 pixels each) to a 2D Gaussian with
 * implicit amplitudes by damped Levenberg-Marquardt, as described by
 * Leutenegger & Weber, "Least-squares fitting of Gaussian spots on graphics
 * processing units":
 *   model      h_i = alpha_hat(p) f_i(p) + beta_hat(p) (Eqs. 2-3); only the
 *              shaping parameters p are iterated
 *   amplitudes closed form of the 2x2 normal equations (Eqs. 5-6)
 *   derivatives of the amplitudes and the residuals (Eqs. 7-9)
 *   profiles   symmetric Gaussian p = (x, y, sigma) (Eqs. 10-11), or
 *              axis-aligned elliptical p = (x, y, sigma_x, sigma_y)
 *   step       (J^T J + lambda diag J^T J) delta = J^T (g - h) (Eqs. 12, 14),
 *              lambda from 0.01, /10 after an improvement, x10 per retry up to
 *              1e4 (Levenberg-Marquardt section); stop rules of the
 *              Fit2DGaussian pseudo-code with the Results-section thresholds.
 *
 * Everything runs on the GPU; this header names no HIP or torch type.  A
 * stream argument is a hipStream_t passed as void* (NULL = the null stream).
 *
 * Pixel data layout (all device memory, caller-owned):
 *   data    uint16 or float32 values; spot s occupies elements
 *           [offsets[s], offsets[s] + w*h), row-major: pixel k = row*w + col
 *           lies at x = col, y = row (0-based pixel centres)
 *   sizes   spotfit_shape_t[n] (w, h, model)
 *   init    float[n][4] = (x, y, sigma_x, sigma_y); symmetric spots read sigma_x
 * Outputs (device, caller-owned, must not alias inputs):
 *   params_out float[n][6] = (x, y, sigma_x, sigma_y, alpha_hat, beta_hat);
 *              symmetric spots report sigma_y = sigma_x
 *   chi2_out   float[n]  raw sum of squared residuals at params_out (the
 *              paper's "normalized" chi^2 is left to the caller, e.g.
 *              chi2 / (w*h - n_params - 2))
 *   iters_out  int32[n]  LM iterations started
 *   status_out int32[n]  spotfit_status_t
 *   evals_out  int32[n][2] or NULL: (derivative evaluations, trial evaluations)
 *
 * Error behaviour: a call returns SPOTFIT_OK or a negative spotfit_error_t.
 * Call-level problems (NULL handle or array, n < 0, invalid options) are
 * detected on the host before any HIP call; n == 0 is a no-op.  Spot-level
 * problems never fail the call: a spot with w or h < 3, w*h above the
 * capacity (1024, or opt.max_pixels when smaller), an unknown model, a
 * non-finite start value or a start width <= 0, or w or h above opt.max_side, gets
 * status SPOTFIT_BAD_INPUT,
 * NaN params and chi^2, and 0 iterations.
 *
 * Asynchrony: work is enqueued on the stream and the call returns; results
 * are valid after the stream is synchronised.  Calls on one context are not
 * thread-safe against each other, and must not overlap on the device: the
 * double-precision kernel hands spots out through a counter the context owns
 * (and the mixed schedule through its workspace), so concurrent streams each
 * need their own context (as the serving loop keeps one per stream).
 */
#ifndef SPOTFIT_H
#define SPOTFIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spotfit_ctx spotfit_ctx_t; /* opaque: device properties, kernel plans */

typedef enum { SPOTFIT_U16 = 0, SPOTFIT_F32 = 1 } spotfit_dtype_t;
typedef enum { SPOTFIT_SYM = 0, SPOTFIT_ELL = 1 } spotfit_model_t;

/* Per-spot stop condition (Fit2DGaussian pseudo-code; the paper leaves the codes unnamed). */
typedef enum {
  SPOTFIT_MAX_ITER = 0,      /* iteration budget used up after an accepted step          */
  SPOTFIT_MAX_ERROR = 1,     /* chi^2 below max_error_per_px * w*h                       */
  SPOTFIT_MIN_DELTA = 2,     /* chi*(1 - min_delta) < Chi: too small an improvement      */
  SPOTFIT_MIN_STEP = 3,      /* every |delta_j| < min_step_rel * |p_j - o_j| (o: below)  */
  SPOTFIT_NOT_CONVERGED = 4, /* NaN error, or no decrease after the damping retries;
                                the parameters before the failed step are returned    */
  SPOTFIT_BAD_INPUT = 5      /* spot-level input error, see above                       */
} spotfit_status_t;

/* Arithmetic of the fit kernel. */
typedef enum {
  SPOTFIT_PREC_FP32 = 0,  /* per-pixel profile kernel, single precision everywhere (the
                             paper's arithmetic)                                        */
  SPOTFIT_PREC_MIXED = 1, /* per-pixel profile kernel: FP32 profile and derivative sums,
                             double-precision parameters, amplitude determinant,
                             residual, chi^2 accumulation and LM solve                  */
  SPOTFIT_PREC_FP64 = 2,  /* default: separable kernel, the profile factors into
                             exp(column) * exp(row); every evaluation in double
                             precision, so chi^2 comparisons see ~1e-15 relative error */
  SPOTFIT_PREC_FP32_PLAIN = 3, /* the paper's own mapping as a baseline: one thread per
                             pixel, one workgroup per spot, one sum per quantity,
                             single precision everywhere                               */
  SPOTFIT_PREC_COMP = 4   /* per-pixel profile kernel as MIXED, but every per-lane sum of
                             an evaluation is compensated: the rounding error of each
                             product (by fma) and of each addition (TwoSum) is carried
                             in a second float, and the lane totals are combined in
                             double; FP32 profile, FP64 determinant and LM solve      */
} spotfit_precision_t;

/* How the separable kernel maps a batch onto lane groups. */
typedef enum {
  SPOTFIT_SCHEDULE_UNIFORM = 0, /* one group width for the whole batch, chosen by max_side;
                                   spots are strided over a persistent grid            */
  SPOTFIT_SCHEDULE_MIXED = 1    /* batches of uneven sizes: a classify pass buckets spots
                                   by size class (largest side <= 8, <= 16, <= 32), then
                                   one persistent launch runs each class with its own
                                   group width; needs the context workspace (see
                                   spotfit_ctx_reserve)                                 */
} spotfit_schedule_t;

/* Which lane mapping the double-precision kernel uses. */
typedef enum {
  SPOTFIT_PLAN_THROUGHPUT = 0, /* default: the most spots per second for batches that fill
                                  the GPU.  Spots up to 16x16 px: 4-lane groups that fit 4
                                  spots at once, one per lane; larger spots: 16-lane groups
                                  of 4 spots.  A batch too small to give every resident spot
                                  slot 1.5-2.5 spots (about 200k-330k spots up to 16 px, 80k
                                  above, on 256 CUs) takes 4 or 16 lanes per spot instead
                                  (the same bits)                                        */
  SPOTFIT_PLAN_LATENCY = 1     /* one lane per column (8, 16 or 32 lanes per spot): each
                                  evaluation step is shorter, so a batch too small to
                                  fill the GPU (a camera frame) finishes sooner; results
                                  agree with the other plan in every decision but may
                                  differ in the last bits                               */
} spotfit_plan_hint_t;

typedef enum {
  SPOTFIT_OK = 0,
  SPOTFIT_E_NULL = -1,     /* NULL context, output or input array with n > 0           */
  SPOTFIT_E_ARG = -2,      /* n < 0, unknown dtype                                       */
  SPOTFIT_E_OPTIONS = -3,  /* options out of range                                       */
  SPOTFIT_E_HIP = -4,      /* a HIP runtime call failed (message via spotfit_last_error) */
  SPOTFIT_E_DEVICE = -5,   /* no usable gfx950 device                                    */
  SPOTFIT_E_AGAIN = -6     /* serving: frame not admitted now (memory or slots); retry   */
} spotfit_error_t;

typedef struct {
  uint8_t w, h;      /* ROI width (columns) and height (rows), 3..32 each, w*h <= 1024 */
  uint8_t model;     /* spotfit_model_t                                                */
  uint8_t reserved;  /* 0                                                              */
} spotfit_shape_t;

typedef struct {
  int32_t max_iter;         /* iteration budget, >= 0 (paper: 20)                          */
  int32_t lambda0_exp10;    /* initial damping 10^k0 (paper: 0.01 -> -2)                   */
  int32_t lambda_max_exp10; /* retry while k < this (paper: 1e4 -> 4)                      */
  int32_t precision;        /* spotfit_precision_t                                          */
  double max_error_per_px;  /* MaxError iff chi^2 < this * w*h (paper "A/3" -> 1/3)        */
  double min_delta;         /* MinDelta iff chi*(1 - min_delta) < Chi (paper: 1e-6)         */
  double min_step_rel;      /* MinStep iff all |delta_j| < this * |p_j - o_j| (paper: 1e-4),
                               o_j = the ROI centre ((w-1)/2, (h-1)/2) for x and y, 0 for
                               the widths (Number of iterations section: < 1 % of the
                               Fig. 8 fits stop on this test)                              */
  double tie_tau;           /* chi^2 changes within +-tie_tau*chi count as ties: neither
                               "improved" nor "worse"; 0 = the paper's exact comparisons  */
  double sigma_min;         /* parameter box of limit(): sigma >= sigma_min (0.3)          */
  double sigma_max_frac;    /* ... sigma <= sigma_max_frac * max(w, h) (1.0); x in
                               [-0.5, w-0.5], y in [-0.5, h-0.5]                           */
  int32_t max_pixels;       /* capacity promise: spots with w*h > max_pixels are
                               BAD_INPUT; smaller values select leaner kernels (1024)     */
  int32_t max_side;         /* capacity promise: spots with w or h > max_side are
                               BAD_INPUT; smaller values select narrower lane groups (32) */
  int32_t schedule;         /* SPOTFIT_PREC_FP64 only: spotfit_schedule_t (UNIFORM)        */
  int32_t plan_hint;        /* SPOTFIT_PREC_FP64 only: spotfit_plan_hint_t (THROUGHPUT)      */
} spotfit_options_t;

/* Fill *opt with the paper's settings (Results section) and the defaults above. */
void spotfit_default_options(spotfit_options_t* opt);

/* SPOTFIT_OK if the options are usable, SPOTFIT_E_OPTIONS otherwise.  Host only. */
int spotfit_validate_options(const spotfit_options_t* opt);

/* Create a context on HIP device `device` (makes it current).  *ctx is owned by
 * the caller and released with spotfit_ctx_destroy.  Returns SPOTFIT_E_DEVICE if
 * the device is not gfx950. */
int spotfit_ctx_create(spotfit_ctx_t** ctx, int device);
void spotfit_ctx_destroy(spotfit_ctx_t* ctx);

/* Size the context's device workspace for mixed-schedule calls of up to n_spots
 * spots (12 bytes per spot plus 544 bytes).  A mixed-schedule call with more spots
 * than reserved grows the workspace itself (one synchronous device allocation),
 * so callers that must not allocate inside a call (graph capture, serving loops)
 * reserve first.  Returns SPOTFIT_OK, SPOTFIT_E_NULL, SPOTFIT_E_ARG or
 * SPOTFIT_E_HIP. */
int spotfit_ctx_reserve(spotfit_ctx_t* ctx, int64_t n_spots);

/* Fit n_spots spots (see the layout above) on `stream`.  All array arguments
 * are device pointers; opt is a host pointer (NULL = defaults).  Allocates
 * nothing, except that a mixed-schedule call on more spots than the context has
 * reserved grows its workspace first (spotfit_ctx_reserve).  Returns SPOTFIT_OK
 * or a negative spotfit_error_t. */
int spotfit_fit_spots(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                      const spotfit_shape_t* sizes, const int64_t* offsets, const float* init,
                      int64_t n_spots, const spotfit_options_t* opt, float* params_out,
                      float* chi2_out, int32_t* iters_out, int32_t* status_out,
                      int32_t* evals_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call, arguments and results as spotfit_fit_spots (bit for bit, with the same
 * context and options), but the fit's scratch memory -- the spot counter of
 * the uniform schedule, the counters and size-class lists of the mixed
 * schedule -- is a fixed array of the library in device memory instead of the
 * context's workspace.  The array is 4 * (200 + 3 * SPOTFIT_NOALLOC_MAX_SPOTS)
 * bytes (about 12.6 MB) on every GPU the library runs on, held until the
 * process ends; its address on a device is looked up when the first context
 * on that device is created.  The call allocates nothing and never grows the
 * context's workspace.  Mixed schedule: at most SPOTFIT_NOALLOC_MAX_SPOTS
 * spots per call (SPOTFIT_E_ARG beyond, checked before any HIP call); the
 * uniform schedule and the single-precision kernels take any n_spots.  Each
 * call clears the counters it uses with a kernel on `stream` before the fit.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (on other streams, from other contexts or host threads) race on it
 * and give wrong results; the caller orders them (calls on one stream are
 * ordered by the stream).  Returns SPOTFIT_OK or a negative spotfit_error_t. */
#define SPOTFIT_NOALLOC_MAX_SPOTS (1 << 20)
int spotfit_fit_spots_noalloc(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                              const spotfit_shape_t* sizes, const int64_t* offsets,
                              const float* init, int64_t n_spots, const spotfit_options_t* opt,
                              float* params_out, float* chi2_out, int32_t* iters_out,
                              int32_t* status_out, int32_t* evals_out, void* stream);

/* Start values on the device, so that raw spots go in and fits come out
 * without a host round trip (the paper takes start values as given and leaves
 * them out of its timings, Results section).  The estimate: background b0 =
 * median of the border ring (top and bottom rows, left and right columns
 * without the corners; the mean of the two middle values), weights
 * max(g - b0, 0), centre = weighted centroid, var_x = sum w (x - cx)^2 / sum w
 * (var_y alike); symmetric sigma = sqrt((var_x + var_y) / 2), elliptical
 * sigma_x = sqrt(var_x), sigma_y = sqrt(var_y); sigmas clamped to
 * [0.8, max(w, h) / 4]; a spot with no pixel above b0 starts at the ROI centre
 * with sigma 1.5.  Writes init_out float[n][4] (device, caller-owned) on
 * `stream`, ready for spotfit_fit_spots; spots that a fit with these options
 * would reject (shape beyond opt->max_side / max_pixels, w or h < 3, unknown
 * model) get NaN.  opt NULL = defaults.  Allocates nothing.  Returns
 * SPOTFIT_OK or a negative spotfit_error_t (checked on the host first). */
int spotfit_moment_init(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                        const spotfit_shape_t* sizes, const int64_t* offsets, int64_t n_spots,
                        const spotfit_options_t* opt, float* init_out, void* stream);

/* The start values the paper uses for its accuracy runs (Results section):
 * the image smoothed by a 3 x 3 moving average (each pixel: the mean of the
 * window pixels that lie inside the ROI), the centre put on the smoothed
 * pixel with the highest value (on ties the first in row-major order),
 * beta0 = lowest raw pixel, alpha0 = highest raw pixel - beta0, and
 * sigma = sqrt(M / pi) with M the number of raw pixels whose value exceeds
 * alpha0 exp(-1/2) + beta0 (formed with one rounding, in double); sigma is at
 * least 0.5 (a flat spot has M = 0).  init_out[s] = (x0, y0, sigma, sigma)
 * for either model.  Window sums are taken in double and are exact for 16-bit
 * pixels (and for float pixels within 2^26 of each other), so the brightest
 * pixel does not depend on the order of additions.  Arguments, unusable
 * shapes (NaN), ownership, stream and return codes as spotfit_moment_init. */
int spotfit_peak_init(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                      const spotfit_shape_t* sizes, const int64_t* offsets, int64_t n_spots,
                      const spotfit_options_t* opt, float* init_out, void* stream);

/* Raw spots in, fits out, in one launch: the start values of
 * spotfit_moment_init and the fit from them (the paper leaves start values to
 * the caller, Results section; its fit is the Fit2DGaussian algorithm with
 * Eqs. 5-14).  With opt->precision SPOTFIT_PREC_FP64 and a batch that the
 * narrow or wide plans fit (the latency hint, or too few spots for the
 * lane-owned plans of SPOTFIT_PLAN_THROUGHPUT), the fit kernel's own lane
 * groups compute each spot's start values before they fit it, so no
 * start-value pass and no round trip through memory sits between frame and
 * fit; a batch that takes a lane-owned plan, and the other precisions, get a
 * start-value launch first (for the lane-owned plans the faster way).
 * init_out float[n][4] (device, caller-owned, required) receives the start
 * values each fit began from (NaN for the shapes spotfit_moment_init rejects,
 * whose fits end as BAD_INPUT).  They equal spotfit_moment_init's up to the
 * order of its double-precision sums (bit for bit where the fit's lanes per
 * spot match the start-value kernel's: the default plans of the uniform
 * schedule), and the fit outputs are bit for bit those of spotfit_fit_spots
 * with init = init_out and the same plan.  The other arguments, ownership,
 * stream and return codes as spotfit_fit_spots. */
int spotfit_fit_raw(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                    const spotfit_shape_t* sizes, const int64_t* offsets, int64_t n_spots,
                    const spotfit_options_t* opt, float* init_out, float* params_out,
                    float* chi2_out, int32_t* iters_out, int32_t* status_out,
                    int32_t* evals_out, void* stream);

/* Stop reasons and iteration counts of a fitted batch: the statistics the
 * paper reports in its Number of iterations section (Fig. 8). */
typedef struct {
  int64_t n_spots;
  int64_t status_count[6];  /* spots per spotfit_status_t                         */
  int64_t iters_hist[65];   /* spots per iteration count 0..63; [64]: 64 or more  */
  int64_t grad_evals;       /* totals over evals_out (0 when it is NULL)          */
  int64_t trial_evals;
} spotfit_stats_t;

/* Summarise the device arrays status[n], iters[n] and evals[n][2] (evals may be
 * NULL) of a fit enqueued earlier on `stream`: a histogram kernel runs on the
 * stream, then the call waits for the stream and fills *out (host).  Uses a
 * buffer the context owns.  Returns SPOTFIT_OK, SPOTFIT_E_NULL, SPOTFIT_E_ARG
 * (n < 0) or SPOTFIT_E_HIP. */
int spotfit_get_stats(spotfit_ctx_t* ctx, const int32_t* status, const int32_t* iters,
                      const int32_t* evals, int64_t n_spots, spotfit_stats_t* out, void* stream);

/* Which lane mapping the autotuner timed and which it kept. */
typedef struct {
  int32_t schedule;      /* spotfit_schedule_t that was tuned                       */
  int32_t size_class;    /* uniform: 0 (max_side <= 8), 1 (<= 16), 2 (<= 32); mixed: -1 */
  int32_t n_candidates;  /* entries used in plan_id / plan_ms                        */
  int32_t chosen;        /* index of the kept plan in plan_id                        */
  int32_t plan_id[16];   /* internal plan numbers (the SPOTFIT_GROUP_PLAN /
                            SPOTFIT_MIXED_PLAN override values)                      */
  double plan_ms[16];    /* mean time of one fit call with that plan                 */
} spotfit_tune_report_t;

/* Autotune the separable double-precision kernel on a representative batch
 * (arguments as for spotfit_fit_spots; opt->precision must be
 * SPOTFIT_PREC_FP64).  Every compiled lane mapping that can hold the batch is
 * timed: for the uniform schedule, the plans whose group holds spots of
 * opt->max_side; for the mixed schedule, the mixed-size plans.  Each plan gets
 * one warm-up call and `reps` (>= 1) timed calls on `stream`, which the call
 * waits for; the fastest is kept in the context for later calls with that
 * schedule and size class.  The output arrays hold the last call's results.
 * All plans take the same decisions on every spot, but their sums run in
 * different orders, so results can differ in the last bits between plans: a
 * context is bitwise reproducible between tunings.  report may be NULL.
 * Returns SPOTFIT_OK or a negative spotfit_error_t. */
int spotfit_autotune(spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                     const spotfit_shape_t* sizes, const int64_t* offsets, const float* init,
                     int64_t n_spots, const spotfit_options_t* opt, float* params_out,
                     float* chi2_out, int32_t* iters_out, int32_t* status_out, int32_t reps,
                     spotfit_tune_report_t* report, void* stream);

/* ------------------------------------------------------------------------ */
/* Captured fits of fixed-shape batches (HIP graphs).                        */
/* ------------------------------------------------------------------------ */
typedef struct spotfit_graph spotfit_graph_t; /* opaque */

/* Optional host side of a captured fit; every pointer is PINNED host memory
 * (hipHostMalloc) or NULL (that copy is left out of the graph). */
typedef struct {
  const void* data;        /* data_bytes bytes copied to the device `data` first   */
  int64_t data_bytes;
  const float* init;       /* n x 4 start values copied to the device `init` first */
  float* params;           /* results copied back after the fit: n x 6             */
  float* chi2;             /* n                                                     */
  int32_t* iters;          /* n                                                     */
  int32_t* status;         /* n                                                     */
} spotfit_graph_io_t;

/* Record one fit of a fixed batch (arguments as spotfit_fit_spots: device
 * arrays, host opt) into a HIP graph, with the host copies `io` names before
 * and after it (io may be NULL), for camera frames whose spot shapes stay the
 * same from frame to frame: the caller refills the inputs (device arrays, or
 * the pinned host buffers of io) and replays the whole call with one
 * spotfit_graph_launch.  The capture runs on a private stream and launches
 * nothing.  The mixed schedule's workspace (12 bytes per spot plus 32) belongs
 * to the graph: allocated here, freed in spotfit_graph_destroy, so later calls
 * on the context (which may grow the context's own workspace) leave it alone.
 * Replays use the context's spot counter: do not overlap them with other calls
 * on the same context.  init may be NULL: the graph then computes the start values on
 * the device as spotfit_fit_raw does (inside the fit's launch for the
 * double-precision kernels), into a buffer of n x 4 floats it allocates here
 * and frees in spotfit_graph_destroy, so that a replay takes raw pixels to
 * fits (io->init must then be NULL).  n_spots must be > 0.  Returns SPOTFIT_OK
 * or a negative spotfit_error_t. */
int spotfit_graph_create(spotfit_graph_t** g, spotfit_ctx_t* ctx, const void* data, int32_t dtype,
                         const spotfit_shape_t* sizes, const int64_t* offsets, const float* init,
                         int64_t n_spots, const spotfit_options_t* opt, float* params_out,
                         float* chi2_out, int32_t* iters_out, int32_t* status_out,
                         const spotfit_graph_io_t* io);
/* Replay the captured call on `stream` (results valid after a stream sync). */
int spotfit_graph_launch(spotfit_graph_t* g, void* stream);
void spotfit_graph_destroy(spotfit_graph_t* g);

/* ------------------------------------------------------------------------ */
/* Serving loop for camera frames (real-time tracking of fiducial spots).    */
/* ------------------------------------------------------------------------ */
typedef struct spotfit_serve spotfit_serve_t; /* opaque */

/* Drift of the sample in one tracked frame (see spotfit_serve_track). */
typedef struct {
  float dx, dy;            /* mean of (x - ref_x, y - ref_y) over the counted markers
                              (pixels; NaN when none counts)                          */
  float mean_dx, mean_dy;  /* mean of (dx, dy) over the last `window` tracked frames
                              that counted a marker, this one included (NaN if none)  */
  int32_t n_used;          /* markers counted in this frame                           */
  int32_t n_frames;        /* frames in the window mean                               */
} spotfit_drift_t;

/* One camera frame, all pointers HOST memory.  Spots lie back to back in `data`
 * (row-major each, no offsets array).  The input buffers may be reused as soon
 * as submit returns; the output arrays must stay valid until the frame is done. */
typedef struct {
  const void* data;              /* n_spots spots of pixels, dtype below              */
  const spotfit_shape_t* sizes;  /* n_spots shapes                                     */
  const float* init;             /* n_spots x 4 start values, or NULL: computed on the
                                    device as by spotfit_moment_init                   */
  int32_t n_spots;
  int32_t dtype;                 /* spotfit_dtype_t                                    */
  float* params_out;             /* n_spots x 6                                        */
  float* chi2_out;               /* n_spots                                            */
  int32_t* iters_out;            /* n_spots, or NULL                                   */
  int32_t* status_out;           /* n_spots, or NULL                                   */
  spotfit_drift_t* drift_out;    /* NULL, or one record: the frame is a tracked frame
                                    (spotfit_serve_track) and its drift lands here     */
} spotfit_frame_t;

typedef struct {
  uint64_t frames_done, frames_failed, spots_done, batches, rejected;
  double latency_p50_us;         /* arrival -> results in the caller's arrays          */
  double latency_p99_us;
  double latency_max_us;
  double mean_frames_per_batch;  /* continuous batching: frames folded per launch      */
  double wall_s;                 /* first arrival to last completion                   */
} spotfit_serve_stats_t;

/* Create a serving loop on `device` with fit options `opt` (NULL = defaults):
 * device memory for at most `device_mem_budget` bytes of frames in flight
 * (3/4 pixels, each frame's pixels followed by its own records, 44 bytes per
 * spot; 1/4 per-spot records of batches, 68 bytes per spot; plus pinned host
 * mirrors of the same size),
 * at most `max_frames` frames in flight, `n_streams` streams (each with its own
 * context) so that batches overlap on the device.  Starts a dispatcher thread. */
int spotfit_serve_create(spotfit_serve_t** sv, int device, const spotfit_options_t* opt,
                         size_t device_mem_budget, int32_t max_frames, int32_t n_streams);

/* Drift tracking of fiducial markers inside the serving loop (the paper's use:
 * marker positions averaged over markers and frames to stabilise the sample,
 * Introduction).  After tracking is set, a frame submitted with drift_out !=
 * NULL must hold exactly n_markers spots, spot k being marker k; right after
 * its fit, on the device, a marker counts when its fit stopped on MAX_ERROR,
 * MIN_DELTA or MIN_STEP with finite x and y, the frame's drift is the mean of
 * (x - ref_x, y - ref_y) over the counted markers (in ROI pixel coordinates,
 * summed in double), and the tracked drift is the mean of the frame drifts of
 * the last `window` tracked frames that counted a marker (in submission order).
 * ref_xy: HOST float[n_markers][2], copied.  n_markers in [1, 65536], window
 * in [1, 65536]; n_markers = 0 turns tracking off.  Allocates device memory
 * for the reference and history; restarts the sequence.  Call it with no frame
 * in flight: otherwise SPOTFIT_E_AGAIN.  Returns SPOTFIT_OK or a negative
 * spotfit_error_t. */
int spotfit_serve_track(spotfit_serve_t* sv, int32_t n_markers, const float* ref_xy,
                        int32_t window);

/* Submit a frame; `arrival_ns` is its arrival time on the steady clock in ns
 * (0 = now), from which its latency is measured.  Returns SPOTFIT_OK and a
 * ticket, or SPOTFIT_E_AGAIN when memory or slots are short (nothing queued).
 * A frame with drift_out but tracking off or a spot count other than the
 * tracked marker count: SPOTFIT_E_ARG. */
int spotfit_serve_submit(spotfit_serve_t* sv, const spotfit_frame_t* frame, uint64_t arrival_ns,
                         uint64_t* ticket);

/* 0 when the frame's results are in its arrays, 1 while pending, < 0 on error:
 * SPOTFIT_E_HIP for a frame whose batch failed (its arrays are not written),
 * for as long as the server lives, also after its ring space is reused.  For
 * tests of this handling, the environment variable SPOTFIT_SERVE_FAIL_BATCH=k
 * read by spotfit_serve_create makes the k-th batch fail on the host, before
 * anything of it is enqueued. */
int spotfit_serve_poll(spotfit_serve_t* sv, uint64_t ticket);
/* Block until the frame is done; SPOTFIT_OK or < 0 on error. */
int spotfit_serve_wait(spotfit_serve_t* sv, uint64_t ticket);
int spotfit_serve_stats(spotfit_serve_t* sv, spotfit_serve_stats_t* out);
/* Stop the dispatcher (frames already launched complete), free everything. */
void spotfit_serve_destroy(spotfit_serve_t* sv);

/* Benchmark driver: submit frames[f] at arrival_offset_ns[f] after a start time
 * (busy-waiting on the steady clock; a refused frame is retried and keeps its
 * arrival time), then wait for all.  Latencies are in spotfit_serve_stats. */
int spotfit_serve_replay(spotfit_serve_t* sv, const spotfit_frame_t* frames, int64_t n_frames,
                         const uint64_t* arrival_offset_ns);

/* Text of the last serving error on this thread.  Host only. */
const char* spotfit_serve_last_error(void);

/* Text of the last error on this thread ("" if none).  Host only. */
const char* spotfit_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int spotfit_version(void);

/* The exponential the double-precision kernels evaluate the profile factors of
 * Eq. 10 with (arguments x <= 0: Cody-Waite reduction by ln 2, Taylor series of
 * degree 13, scaling by 2^n), applied elementwise: y[i] = e^x[i] for the n
 * device doubles x, written to the device array y, on `stream`.  For accuracy
 * tests against a reference exponential.  x > 0 is outside its range.  Returns
 * SPOTFIT_OK, SPOTFIT_E_NULL, SPOTFIT_E_ARG (n < 0) or SPOTFIT_E_HIP. */
int spotfit_exp_neg(const double* x, double* y, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SPOTFIT_H */
