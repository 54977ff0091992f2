/*
 * spotfit_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, double-precision CPU reference of the implicit-amplitude
 * Levenberg-Marquardt fit of 2D Gaussian spots (Leutenegger & Weber,
 * "Least-squares fitting of Gaussian spots on graphics processing units").
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may call it.  It shares no code, header, table or helper with the HIP path.
 *
 * Parity status per function (what pins it; see the tests):
 *   orc_eval   Eqs. 5-6 pinned to a textbook linear least-squares solve,
 *              Eqs. 7-9 and 11 pinned to central finite differences,
 *              the gradient pinned to the envelope identity.
 *   orc_solve  pinned to a generic dense solve of the damped system (Eq. 14).
 *   orc_fit_*  pinned by noise-free recovery, by equality with an explicit
 *              five-parameter least-squares fit (scipy), by brute-force grid
 *              search on tiny spots, statistically by Table 1 / Fig. 8, and
 *              in its control flow by replaying the logged trajectory
 *              (orc_fit_spot_traced) against the pseudo-code with chi^2, the
 *              Jacobian and the damped step computed independently in the
 *              tests, through every exit: the damping cap with the best point
 *              restored, MaxError before and after a trial, MinDelta, MinStep,
 *              and the iteration budget.
 *   The status codes, the MaxError threshold "A/3", the limit() box and the
 *   chi^2 normalisation are the paper's unspecified details: parity unpinned.
 *   orc_moment_init  (start values, outside the paper's method) pinned by
 *              hand-built images with known centroid / moments, the flat and
 *              single-pixel degenerate cases, and an independent vectorised
 *              implementation of the same estimate.
 *   orc_peak_init  (the paper's start values, Results section) pinned by a
 *              lone bright pixel (window ties), a flat image, plateaus of known
 *              area, a library 2-D convolution with first-occurrence argmax,
 *              and the Table 1 statistics it feeds.
 */
#ifndef SPOTFIT_ORACLE_H
#define SPOTFIT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SYM = 0, ORC_ELL = 1 };
enum { ORC_MAX_ITER = 0, ORC_MAX_ERROR = 1, ORC_MIN_DELTA = 2, ORC_MIN_STEP = 3,
       ORC_NOT_CONVERGED = 4, ORC_BAD_INPUT = 5 };

typedef struct {
  int32_t max_iter;          /* iteration budget (paper: 20)                          */
  double  max_error_per_px;  /* MaxError iff chi^2 < max_error_per_px * N  ("A/3")    */
  double  min_delta;         /* MinDelta iff chi*(1-min_delta) < Chi   (paper: 1e-6)  */
  double  min_step_rel;      /* MinStep iff all |delta_j| < min_step_rel*|p_j - o_j|, o = ROI centre for x, y (1e-4) */
  int32_t lambda0_exp10;     /* initial damping 10^k0 (paper: 0.01 -> -2)             */
  int32_t lambda_max_exp10;  /* retries while k < this (paper: 10^4 -> 4)             */
  double  tie_tau;           /* relative tie band for chi^2 comparisons (0 = verbatim) */
  double  sigma_min;         /* limit(): sigma >= sigma_min                           */
  double  sigma_max_frac;    /* limit(): sigma <= sigma_max_frac * max(w, h)          */
} orc_opts;

typedef struct {
  double  params[6];   /* x, y, sigma_x, sigma_y, alpha, beta (sym: sigma_y = sigma_x) */
  double  chi2;        /* raw sum of squared residuals at params                        */
  int32_t iters;       /* loop passes started                                          */
  int32_t status;      /* ORC_* code                                                   */
  int32_t n_grad;      /* evaluations with derivatives                                 */
  int32_t n_trial;     /* evaluations without derivatives (trial steps)               */
  double  margin_chi;  /* smallest relative margin of any chi^2 comparison taken       */
  double  margin_step; /* smallest relative margin of any step-size comparison taken   */
  double  min_pivot;   /* smallest pivot / diagonal ratio of any damped solve (1 = none;
                          near 0: an ill-conditioned step that rounding can move far)  */
} orc_result;

void orc_default_opts(orc_opts* o);

/* Number of shaping parameters of a model (3 or 4), or 0 if unknown. */
int orc_nparams(int model);

/* One evaluation of the reduced model at shaping parameters p (Eqs. 2-11).
 * g: w*h pixel values (row-major), p: n shaping params.
 * out3 = (alpha_hat, beta_hat, chi^2).  If want_grad: A (n*n, row-major) = J^T J,
 * bvec (n) = J^T (g - h) and, when J != NULL, J (N*n) = d r_k / d p_j with
 * r = h - g.  Returns 0, or 1 when N*sum f^2 - (sum f)^2 is not positive or the
 * result is not finite (then chi^2 = NaN). */
int orc_eval(const double* g, int w, int h, int model, const double* p, int want_grad,
             double* out3, double* A, double* bvec, double* J);

/* Damped step (Eq. 14): (A + lam*diag(A)) delta = bvec by Cholesky.
 * Returns 0, or 1 (delta set to NaN) if the matrix is not positive definite. */
int orc_solve(const double* A, const double* bvec, int n, double lam, double* delta);

/* 10^k from its definition (exact for |k| <= 22). */
double orc_pow10(int k);

/* Whole fit of one spot from init4 = (x, y, sigma_x, sigma_y). */
void orc_fit_spot(const double* g, int w, int h, int model, const float* init4,
                  const orc_opts* o, orc_result* res);

/* One evaluation of the Levenberg-Marquardt loop, in the order the loop takes
 * them: the evaluation with derivatives that opens iteration `iter` (GRAD), the
 * first trial of that iteration (TRIAL) and each retry with more damping
 * (RETRY).  k is the damping exponent in force (for a trial: the one its step
 * was solved with), p the point evaluated (a trial's is limit(best + delta)),
 * delta the unclamped step of a trial (0 for GRAD), chi its chi^2 (NaN when
 * the evaluation failed). */
enum { ORC_EV_GRAD = 0, ORC_EV_TRIAL = 1, ORC_EV_RETRY = 2 };
typedef struct {
  int32_t kind, iter, k, pad;
  double  p[4];
  double  delta[4];
  double  chi;
} orc_event;

/* orc_fit_spot that also logs its trajectory: up to cap events into ev, their
 * total count (which may exceed cap) into *n_ev.  ev may be NULL. */
void orc_fit_spot_traced(const double* g, int w, int h, int model, const float* init4,
                         const orc_opts* o, orc_result* res, orc_event* ev, int cap,
                         int* n_ev);

/* Batch driver over the ragged layout; dtype 0 = uint16, 1 = float32.
 * Every output array has n entries (params: n*6).  Spots are split into
 * contiguous static chunks over n_threads POSIX threads. Returns 0 or -1. */
int orc_fit_batch(const void* data, int dtype, const uint8_t* sizes, const int64_t* offsets,
                  const float* init, int64_t n, const orc_opts* o, double* params,
                  double* chi2, int32_t* iters, int32_t* status, int32_t* n_grad,
                  int32_t* n_trial, double* margin_chi, double* margin_step,
                  double* min_pivot, int n_threads);

/* Centroid / second-moment start values of one spot (row-major g, w x h):
 * background = median of the border ring, weights max(g - b0, 0), weighted
 * centroid and variances, sigmas clamped to [0.8, max(w, h) / 4]; no positive
 * weight: ROI centre, sigma 1.5.  out = (x, y, sigma_x, sigma_y); returns 0,
 * or -1 (NaN out) for w or h < 3, more than 1024 pixels or an unknown model. */
int orc_moment_init(const double* g, int w, int h, int model, double* out);

/* The same for a ragged batch in the library's layout; out double[n][4]. */
int orc_moment_init_batch(const void* data, int dtype, const uint8_t* sizes,
                          const int64_t* offsets, int64_t n, double* out);

/* The paper's start values (Results section): centre = brightest pixel of the
 * 3 x 3 moving average (mean over the in-ROI part of the window; first in
 * row-major order on ties); sigma = sqrt(M / pi), M = raw pixels above
 * (max - min) exp(-1/2) + min (fused multiply-add), at least 0.5.  out = (x, y,
 * sigma, sigma); returns 0, or -1 (NaN out) for w or h < 3 or more than 1024
 * pixels. */
int orc_peak_init(const double* g, int w, int h, double* out);
int orc_peak_init_batch(const void* data, int dtype, const uint8_t* sizes,
                        const int64_t* offsets, int64_t n, double* out);

#ifdef __cplusplus
}
#endif
#endif
