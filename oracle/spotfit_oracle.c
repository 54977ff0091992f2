/*
 * spotfit_oracle.c -- TEST INFRASTRUCTURE ONLY: the double-precision CPU
 * reference the HIP path is checked against.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark may call it; the product path never
 * does.  Plain serial C, one spot at a time, double throughout, libm exp(), no
 * blocking, fusion or reordering beyond what the paper's equations state.
 *
 * Method (Leutenegger & Weber, Method section):
 *   model      h_i = alpha f_i(p) + beta, p = shaping parameters only (Eq. 2)
 *   profile    symmetric Gaussian (Eq. 10) with derivatives (Eq. 11); the
 *              axis-aligned elliptical variant uses the same construction with
 *              one width per axis
 *   amplitudes closed-form alpha_hat, beta_hat of the inner 2x2 least squares
 *              (Eqs. 3-6)
 *   Jacobian   d alpha_hat / d p_j and d beta_hat / d p_j (Eqs. 7-8) give the
 *              derivative of each residual, the second factor of Eq. 9
 *   step       damped normal equations (Eqs. 12, 14), lambda schedule and stop
 *              rules of the Levenberg-Marquardt section and the Fit2DGaussian
 *              pseudo-code, with the iteration budget and thresholds of the
 *              Results section.
 *
 * Readings of points the paper leaves open (each is also used by the HIP path,
 * implemented there independently):
 *   - Eq. 12's right-hand side is taken as J^T (g - h) with J = dh/dp, so the
 *     step descends; J is the per-pixel residual derivative (Eq. 9's second
 *     factor), the "Hessian" is J^T J.
 *   - Inside the retry loop the re-evaluated error is the trial error Chi.
 *   - lambda = 10^k with an integer exponent k: k0 = -2, k -= 1 after an
 *     improving first trial, retries while k < 4 (lambda up to 1e4).
 *   - MaxError uses A = number of pixels: chi^2 < max_error_per_px * N.
 *   - MinStep is relative: all |delta_j| < min_step_rel * |best_j - o_j|, on
 *     the unclamped step, with the centre coordinates measured from the centre
 *     of the ROI (o = ((w-1)/2, (h-1)/2) for x and y, 0 for the widths): the
 *     reading under which fewer than 1 % of the fits of the paper's Fig. 8 run
 *     stop on this test, as the Number of iterations section states (about
 *     5 % would from the corner pixel's centre, in double and in single
 *     precision alike).
 *   - limit(): x in [-0.5, w-0.5], y in [-0.5, h-0.5],
 *     sigma in [sigma_min, sigma_max_frac*max(w,h)]; NaN passes through.
 *   - tie_tau: chi^2 comparisons "improved" / "worse" use the band
 *     Chi < chi(1-tau) / Chi > chi(1+tau); tau = 0 is the paper verbatim.
 *   - Pixel k = row*w + col sits at x = col, y = row.
 */
#include "spotfit_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXPIX 1024
#define ORC_MAXP 4

void orc_default_opts(orc_opts* o) {
  o->max_iter = 20;               /* Results: limited to 20 iterations        */
  o->max_error_per_px = 1.0 / 3.0; /* Results: chi^2 < A/3                    */
  o->min_delta = 1e-6;            /* Results: decrease below 1e-6 chi^2       */
  o->min_step_rel = 1e-4;         /* Results: |dp_j| < 1e-4 |p_j|             */
  o->lambda0_exp10 = -2;          /* LM section: initial damping 0.01         */
  o->lambda_max_exp10 = 4;        /* LM section: damping beyond 1e4 stops     */
  o->tie_tau = 0.0;
  o->sigma_min = 0.3;
  o->sigma_max_frac = 1.0;
}

int orc_nparams(int model) {
  if (model == ORC_SYM) return 3;
  if (model == ORC_ELL) return 4;
  return 0;
}

double orc_pow10(int k) {
  double t = 1.0;
  int m = k < 0 ? -k : k;
  for (int i = 0; i < m; ++i) t *= 10.0;
  return k < 0 ? 1.0 / t : t;
}

/* Profile value and its derivatives with respect to the shaping parameters at
 * pixel (x, y).  Symmetric (Eqs. 10-11): p = (xc, yc, s).  Elliptical: p = (xc,
 * yc, sx, sy), f = exp(-dx^2/(2 sx^2) - dy^2/(2 sy^2)), df/dxc = dx f/sx^2,
 * df/dyc = dy f/sy^2, df/dsx = dx^2 f/sx^3, df/dsy = dy^2 f/sy^3. */
static double profile(int model, const double* p, double x, double y, double* df) {
  double dx = x - p[0], dy = y - p[1];
  if (model == ORC_SYM) {
    double s = p[2];
    double rr = dx * dx + dy * dy;
    double f = exp(-rr / (2.0 * s * s));
    if (df) {
      df[0] = dx / (s * s) * f;
      df[1] = dy / (s * s) * f;
      df[2] = rr / (s * s * s) * f;
    }
    return f;
  } else {
    double sx = p[2], sy = p[3];
    double f = exp(-dx * dx / (2.0 * sx * sx) - dy * dy / (2.0 * sy * sy));
    if (df) {
      df[0] = dx / (sx * sx) * f;
      df[1] = dy / (sy * sy) * f;
      df[2] = dx * dx / (sx * sx * sx) * f;
      df[3] = dy * dy / (sy * sy * sy) * f;
    }
    return f;
  }
}

int orc_eval(const double* g, int w, int h, int model, const double* p, int want_grad,
             double* out3, double* A, double* bvec, double* J) {
  const int N = w * h;
  const int n = orc_nparams(model);
  double f[ORC_MAXPIX];
  double df[ORC_MAXPIX][ORC_MAXP];

  /* step 1: profile (and its derivatives) at every pixel */
  for (int k = 0; k < N; ++k) {
    double x = (double)(k % w), y = (double)(k / w);
    f[k] = profile(model, p, x, y, want_grad ? df[k] : NULL);
  }

  /* step 2: sums of Eq. 5 and the closed-form amplitudes of Eq. 6 */
  double F = 0.0, G = 0.0, FF = 0.0, FG = 0.0;
  for (int k = 0; k < N; ++k) {
    F += f[k];
    G += g[k];
    FF += f[k] * f[k];
    FG += f[k] * g[k];
  }
  double D = (double)N * FF - F * F;
  out3[0] = out3[1] = out3[2] = NAN;
  if (!(D > 0.0) || !isfinite(D)) return 1;
  double a = ((double)N * FG - F * G) / D;
  double b = (G * FF - F * FG) / D;

  /* step 3: residuals r = h - g and the error of Eq. 2 */
  double chi = 0.0;
  for (int k = 0; k < N; ++k) {
    double r = a * f[k] + b - g[k];
    chi += r * r;
  }
  if (!isfinite(chi) || !isfinite(a) || !isfinite(b)) return 1;
  out3[0] = a;
  out3[1] = b;
  out3[2] = chi;
  if (!want_grad) return 0;

  /* derivative sums of Eq. 7 */
  double dF[ORC_MAXP], dFF[ORC_MAXP], dFG[ORC_MAXP], gam[ORC_MAXP];
  double da[ORC_MAXP], db[ORC_MAXP];
  for (int j = 0; j < n; ++j) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int k = 0; k < N; ++k) {
      s1 += df[k][j];
      s2 += f[k] * df[k][j];
      s3 += g[k] * df[k][j];
    }
    dF[j] = s1;
    dFF[j] = 2.0 * s2;
    dFG[j] = s3;
    gam[j] = (double)N * dFF[j] - 2.0 * F * dF[j];
    /* Eq. 8 */
    da[j] = ((double)N * dFG[j] - G * dF[j] - a * gam[j]) / D;
    db[j] = (G * dFF[j] - FG * dF[j] - F * dFG[j] - b * gam[j]) / D;
  }

  /* residual derivatives (second factor of Eq. 9), normal matrix and gradient */
  for (int i = 0; i < n * n; ++i) A[i] = 0.0;
  for (int j = 0; j < n; ++j) bvec[j] = 0.0;
  for (int k = 0; k < N; ++k) {
    double r = a * f[k] + b - g[k];
    double Jk[ORC_MAXP];
    for (int j = 0; j < n; ++j) {
      Jk[j] = da[j] * f[k] + a * df[k][j] + db[j];
      if (J) J[(size_t)k * n + j] = Jk[j];
    }
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) A[i * n + j] += Jk[i] * Jk[j];
      bvec[i] -= Jk[i] * r;
    }
  }
  return 0;
}

/* Cholesky solve of the damped system; *min_pivot (when not NULL) is lowered to
 * the smallest ratio of a pivot to its diagonal entry, s_j / M_jj in (0, 1]: how
 * much of each diagonal entry survives elimination.  Its reciprocal grows like
 * the condition number of the diagonally scaled matrix, which sets how far
 * rounding in A and b can move delta. */
static int chol_solve(const double* A, const double* bvec, int n, double lam, double* delta,
                      double* min_pivot) {
  double M[ORC_MAXP][ORC_MAXP], L[ORC_MAXP][ORC_MAXP], y[ORC_MAXP];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) M[i][j] = A[i * n + j] + (i == j ? lam * A[i * n + j] : 0.0);
  memset(L, 0, sizeof L);
  for (int j = 0; j < n; ++j) {
    double s = M[j][j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(s > 0.0) || !isfinite(s)) goto fail;
    if (min_pivot && M[j][j] > 0.0 && s / M[j][j] < *min_pivot) *min_pivot = s / M[j][j];
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = M[i][j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  for (int i = 0; i < n; ++i) {
    double t = bvec[i];
    for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
    y[i] = t / L[i][i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = y[i];
    for (int k = i + 1; k < n; ++k) t -= L[k][i] * delta[k];
    delta[i] = t / L[i][i];
  }
  for (int i = 0; i < n; ++i)
    if (!isfinite(delta[i])) goto fail;
  return 0;
fail:
  for (int i = 0; i < n; ++i) delta[i] = NAN;
  return 1;
}

int orc_solve(const double* A, const double* bvec, int n, double lam, double* delta) {
  return chol_solve(A, bvec, n, lam, delta, NULL);
}

static double clampnan(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

static void limit_params(double* p, int model, int w, int h, const orc_opts* o) {
  double smax = o->sigma_max_frac * (double)(w > h ? w : h);
  p[0] = clampnan(p[0], -0.5, (double)w - 0.5);
  p[1] = clampnan(p[1], -0.5, (double)h - 0.5);
  p[2] = clampnan(p[2], o->sigma_min, smax);
  if (model == ORC_ELL) p[3] = clampnan(p[3], o->sigma_min, smax);
}

/* decision bookkeeping: each comparison records how far it was from flipping */
static void note(double* m, double v) {
  if (isfinite(v) && v < *m) *m = v;
}

static int chi_below(double lhs, double rhs, double scale, double* margin) {
  /* lhs < rhs, margin relative to scale */
  if (scale > 0.0) note(margin, fabs(lhs - rhs) / scale);
  return lhs < rhs;
}

/* MinStep: every |d_j| below rel times the size of the parameter, the centre
 * coordinates taken from the centre (cx, cy) of the ROI */
static int all_small(const double* d, const double* best, int n, double rel, double cx,
                     double cy, double* margin) {
  int all = 1;
  for (int j = 0; j < n; ++j) {
    const double org = j == 0 ? cx : (j == 1 ? cy : 0.0);
    double lim = rel * fabs(best[j] - org);
    if (lim > 0.0) note(margin, fabs(fabs(d[j]) - lim) / lim);
    if (!(fabs(d[j]) < lim)) all = 0;
  }
  return all;
}

/* Appends one evaluation of the loop to the trajectory log (when one is kept). */
static void log_eval(orc_event* ev, int cap, int* n_ev, int kind, int iter, int k,
                     const double* p, const double* delta, double chi, int n) {
  if (!ev || !n_ev || *n_ev >= cap) {
    if (n_ev) ++*n_ev;
    return;
  }
  orc_event* e = &ev[*n_ev];
  memset(e, 0, sizeof *e);
  e->kind = kind;
  e->iter = iter;
  e->k = k;
  for (int j = 0; j < n; ++j) {
    e->p[j] = p[j];
    e->delta[j] = delta ? delta[j] : 0.0;
  }
  e->chi = chi;
  ++*n_ev;
}

void orc_fit_spot(const double* g, int w, int h, int model, const float* init4,
                  const orc_opts* o, orc_result* res) {
  orc_fit_spot_traced(g, w, h, model, init4, o, res, NULL, 0, NULL);
}

void orc_fit_spot_traced(const double* g, int w, int h, int model, const float* init4,
                         const orc_opts* o, orc_result* res, orc_event* ev, int cap,
                         int* n_ev) {
  const int n = orc_nparams(model);
  if (n_ev) *n_ev = 0;
  const int N = w * h;
  memset(res, 0, sizeof *res);
  res->margin_chi = INFINITY;
  res->margin_step = INFINITY;
  res->min_pivot = 1.0;
  for (int i = 0; i < 6; ++i) res->params[i] = NAN;
  res->chi2 = NAN;
  res->status = ORC_BAD_INPUT;

  /* spot-level input checks: sizes, model, finite init with positive widths */
  if (n == 0 || w < 3 || h < 3 || N > ORC_MAXPIX) return;
  for (int i = 0; i < n; ++i)
    if (!isfinite((double)init4[i])) return;
  if (!(init4[2] > 0.0f) || (model == ORC_ELL && !(init4[3] > 0.0f))) return;

  const double T = o->max_error_per_px * (double)N;  /* MaxError threshold */
  const double cx = 0.5 * (double)(w - 1), cy = 0.5 * (double)(h - 1);  /* ROI centre */
  const double tau = o->tie_tau;
  double p[ORC_MAXP], best[ORC_MAXP], delta[ORC_MAXP];
  double A[ORC_MAXP * ORC_MAXP], bvec[ORC_MAXP], e3[3];
  for (int i = 0; i < n; ++i) p[i] = (double)init4[i];

  int k = o->lambda0_exp10;
  int it = 0;
  int status = ORC_MAX_ITER;
  double* mc = &res->margin_chi;
  double* ms = &res->margin_step;

  while (it < o->max_iter) {
    ++it;
    orc_eval(g, w, h, model, p, 1, e3, A, bvec, NULL);
    res->n_grad++;
    double chi = e3[2];
    log_eval(ev, cap, n_ev, ORC_EV_GRAD, it, k, p, NULL, chi, n);
    if (isnan(chi)) { status = ORC_NOT_CONVERGED; break; }
    if (chi_below(chi, T, T, mc)) { status = ORC_MAX_ERROR; break; }

    memcpy(best, p, sizeof(double) * n);
    chol_solve(A, bvec, n, orc_pow10(k), delta, &res->min_pivot);
    for (int j = 0; j < n; ++j) p[j] = best[j] + delta[j];
    limit_params(p, model, w, h, o);
    orc_eval(g, w, h, model, p, 0, e3, NULL, NULL, NULL);
    res->n_trial++;
    double Chi = e3[2];
    log_eval(ev, cap, n_ev, ORC_EV_TRIAL, it, k, p, delta, Chi, n);

    /* improved: Chi < chi(1 - tau) -> less damping */
    if (chi_below(Chi, chi * (1.0 - tau), chi, mc)) --k;

    /* retry with more damping while the step is not tiny, the error grew
       (Chi > chi(1 + tau)) and lambda may still grow */
    while (!all_small(delta, best, n, o->min_step_rel, cx, cy, ms) &&
           chi_below(chi * (1.0 + tau), Chi, chi, mc) && k < o->lambda_max_exp10) {
      ++k;
      chol_solve(A, bvec, n, orc_pow10(k), delta, &res->min_pivot);
      for (int j = 0; j < n; ++j) p[j] = best[j] + delta[j];
      limit_params(p, model, w, h, o);
      orc_eval(g, w, h, model, p, 0, e3, NULL, NULL, NULL);
      res->n_trial++;
      Chi = e3[2];
      log_eval(ev, cap, n_ev, ORC_EV_RETRY, it, k, p, delta, Chi, n);
    }

    if (chi_below(chi * (1.0 + tau), Chi, chi, mc) || isnan(Chi)) {
      memcpy(p, best, sizeof(double) * n);
      status = ORC_NOT_CONVERGED;
      break;
    }
    if (chi_below(Chi, T, T, mc)) { status = ORC_MAX_ERROR; break; }
    if (chi_below(chi * (1.0 - o->min_delta), Chi, chi, mc)) { status = ORC_MIN_DELTA; break; }
    if (all_small(delta, best, n, o->min_step_rel, cx, cy, ms)) { status = ORC_MIN_STEP; break; }
  }

  /* final error and amplitudes at the returned parameters */
  orc_eval(g, w, h, model, p, 0, e3, NULL, NULL, NULL);
  res->params[0] = p[0];
  res->params[1] = p[1];
  res->params[2] = p[2];
  res->params[3] = (model == ORC_ELL) ? p[3] : p[2];
  res->params[4] = e3[0];
  res->params[5] = e3[1];
  res->chi2 = e3[2];
  res->iters = it;
  res->status = status;
}

typedef struct {
  const void* data; int dtype; const uint8_t* sizes; const int64_t* offsets; const float* init;
  const orc_opts* o; double* params; double* chi2; int32_t* iters; int32_t* status;
  int32_t* n_grad; int32_t* n_trial; double* margin_chi; double* margin_step;
  double* min_pivot;
  int64_t lo, hi;
} orc_job;

static void* run_job(void* arg) {
  orc_job* jb = (orc_job*)arg;
  double g[ORC_MAXPIX];
  for (int64_t s = jb->lo; s < jb->hi; ++s) {
    int w = jb->sizes[4 * s + 0], h = jb->sizes[4 * s + 1], model = jb->sizes[4 * s + 2];
    int N = w * h;
    orc_result r;
    if (N <= ORC_MAXPIX) {
      if (jb->dtype == 0) {
        const uint16_t* d = (const uint16_t*)jb->data + jb->offsets[s];
        for (int k = 0; k < N; ++k) g[k] = (double)d[k];
      } else {
        const float* d = (const float*)jb->data + jb->offsets[s];
        for (int k = 0; k < N; ++k) g[k] = (double)d[k];
      }
    }
    orc_fit_spot(g, w, h, model, jb->init + 4 * s, jb->o, &r);
    for (int i = 0; i < 6; ++i) jb->params[6 * s + i] = r.params[i];
    jb->chi2[s] = r.chi2;
    jb->iters[s] = r.iters;
    jb->status[s] = r.status;
    if (jb->n_grad) jb->n_grad[s] = r.n_grad;
    if (jb->n_trial) jb->n_trial[s] = r.n_trial;
    if (jb->margin_chi) jb->margin_chi[s] = r.margin_chi;
    if (jb->margin_step) jb->margin_step[s] = r.margin_step;
    if (jb->min_pivot) jb->min_pivot[s] = r.min_pivot;
  }
  return NULL;
}

int orc_fit_batch(const void* data, int dtype, const uint8_t* sizes, const int64_t* offsets,
                  const float* init, int64_t n, const orc_opts* o, double* params,
                  double* chi2, int32_t* iters, int32_t* status, int32_t* n_grad,
                  int32_t* n_trial, double* margin_chi, double* margin_step,
                  double* min_pivot, int n_threads) {
  if (n < 0 || (dtype != 0 && dtype != 1) || !o) return -1;
  if (n == 0) return 0;
  if (!data || !sizes || !offsets || !init || !params || !chi2 || !iters || !status) return -1;
  if (n_threads < 1) n_threads = 1;
  if ((int64_t)n_threads > n) n_threads = (int)n;
  orc_job* jobs = (orc_job*)calloc((size_t)n_threads, sizeof(orc_job));
  pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -1; }
  int64_t per = (n + n_threads - 1) / n_threads;
  for (int t = 0; t < n_threads; ++t) {
    orc_job* jb = &jobs[t];
    jb->data = data; jb->dtype = dtype; jb->sizes = sizes; jb->offsets = offsets;
    jb->init = init; jb->o = o; jb->params = params; jb->chi2 = chi2; jb->iters = iters;
    jb->status = status; jb->n_grad = n_grad; jb->n_trial = n_trial;
    jb->margin_chi = margin_chi; jb->margin_step = margin_step; jb->min_pivot = min_pivot;
    jb->lo = t * per;
    jb->hi = (t + 1) * per < n ? (t + 1) * per : n;
  }
  /* worker threads take chunks 1..T-1; a chunk whose thread cannot start runs here */
  char* started = (char*)calloc((size_t)n_threads, 1);
  for (int t = 1; t < n_threads; ++t)
    if (started && jobs[t].lo < jobs[t].hi)
      started[t] = pthread_create(&th[t], NULL, run_job, &jobs[t]) == 0;
  run_job(&jobs[0]);
  for (int t = 1; t < n_threads; ++t) {
    if (jobs[t].lo >= jobs[t].hi) continue;
    if (started && started[t]) pthread_join(th[t], NULL);
    else run_job(&jobs[t]);
  }
  free(started);
  free(jobs);
  free(th);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Start values from the pixels (not part of the paper's method, which takes */
/* start values as given, Results section): the centroid / second-moment     */
/* estimate.  Background b0 = median of the border ring (top row, bottom row, */
/* then the left and right columns without the corners; an even count, so   */
/* the mean of the two middle values); weights wt = max(g - b0, 0); centre = */
/* the weighted centroid; symmetric sigma^2 = (var_x + var_y) / 2, elliptical */
/* sigma_x^2 = var_x, sigma_y^2 = var_y, with var_x = sum wt (x - cx)^2 /     */
/* sum wt; sigmas clamped to [0.8, max(w, h) / 4]; with no positive weight   */
/* the ROI centre and sigma 1.5.                                             */
/* ------------------------------------------------------------------------ */
int orc_moment_init(const double* g, int w, int h, int model, double* out) {
  for (int i = 0; i < 4; ++i) out[i] = NAN;
  if (w < 3 || h < 3 || w * h > ORC_MAXPIX || orc_nparams(model) == 0) return -1;
  double ring[4 * 32];
  int n = 0;
  for (int c = 0; c < w; ++c) ring[n++] = g[c];
  for (int c = 0; c < w; ++c) ring[n++] = g[(h - 1) * w + c];
  for (int r = 1; r < h - 1; ++r) ring[n++] = g[r * w];
  for (int r = 1; r < h - 1; ++r) ring[n++] = g[r * w + w - 1];
  for (int i = 1; i < n; ++i) { /* insertion sort */
    const double v = ring[i];
    int j = i - 1;
    while (j >= 0 && ring[j] > v) { ring[j + 1] = ring[j]; --j; }
    ring[j + 1] = v;
  }
  const double b0 = 0.5 * (ring[n / 2 - 1] + ring[n / 2]);
  double sw = 0.0, swx = 0.0, swy = 0.0;
  for (int r = 0; r < h; ++r)
    for (int c = 0; c < w; ++c) {
      const double wt = fmax(g[r * w + c] - b0, 0.0);
      sw += wt;
      swx += wt * c;
      swy += wt * r;
    }
  if (!(sw > 0.0)) {
    out[0] = 0.5 * (w - 1);
    out[1] = 0.5 * (h - 1);
    out[2] = out[3] = 1.5;
    return 0;
  }
  const double cx = swx / sw, cy = swy / sw;
  double vx = 0.0, vy = 0.0;
  for (int r = 0; r < h; ++r)
    for (int c = 0; c < w; ++c) {
      const double wt = fmax(g[r * w + c] - b0, 0.0);
      vx += wt * (c - cx) * (c - cx);
      vy += wt * (r - cy) * (r - cy);
    }
  vx /= sw;
  vy /= sw;
  double sx, sy;
  if (model == ORC_SYM) {
    sx = sy = sqrt(0.5 * (vx + vy));
  } else {
    sx = sqrt(vx);
    sy = sqrt(vy);
  }
  const double lo = 0.8, hi = 0.25 * (w > h ? w : h);
  out[0] = cx;
  out[1] = cy;
  out[2] = sx < lo ? lo : (sx > hi ? hi : sx);
  out[3] = sy < lo ? lo : (sy > hi ? hi : sy);
  return 0;
}

int orc_moment_init_batch(const void* data, int dtype, const uint8_t* sizes,
                          const int64_t* offsets, int64_t n, double* out) {
  double g[ORC_MAXPIX];
  for (int64_t s = 0; s < n; ++s) {
    const int w = sizes[4 * s], h = sizes[4 * s + 1], model = sizes[4 * s + 2];
    if (w < 3 || h < 3 || w * h > ORC_MAXPIX) {
      for (int i = 0; i < 4; ++i) out[4 * s + i] = NAN;
      continue;
    }
    for (int k = 0; k < w * h; ++k)
      g[k] = dtype == 0 ? (double)((const uint16_t*)data)[offsets[s] + k]
                        : (double)((const float*)data)[offsets[s] + k];
    orc_moment_init(g, w, h, model, out + 4 * s);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The paper's own start values for its accuracy runs (Results section,      */
/* initial parameters): smooth the image with a 3 x 3 moving average (here   */
/* the mean over the part of the window inside the ROI); the centre is the   */
/* smoothed pixel with the highest value (the first one in row-major order   */
/* on ties); beta0 = lowest raw pixel, alpha0 = highest raw pixel - beta0;   */
/* sigma = sqrt(M / pi) with M the number of raw pixels whose value exceeds  */
/* alpha0 exp(-1/2) + beta0 (that threshold formed with a single rounding);  */
/* sigma is kept >= 0.5 (a flat image has M = 0).  Both sigmas get the same */
/* value.                                                                    */
/* ------------------------------------------------------------------------ */
int orc_peak_init(const double* g, int w, int h, double* out) {
  for (int i = 0; i < 4; ++i) out[i] = NAN;
  if (w < 3 || h < 3 || w * h > ORC_MAXPIX) return -1;
  double best = -INFINITY;
  int bx = 0, by = 0;
  for (int r = 0; r < h; ++r)
    for (int c = 0; c < w; ++c) {
      double acc = 0.0;
      int cnt = 0;
      for (int dr = -1; dr <= 1; ++dr)
        for (int dc = -1; dc <= 1; ++dc) {
          const int rr = r + dr, cc = c + dc;
          if (rr < 0 || rr >= h || cc < 0 || cc >= w) continue;
          acc += g[rr * w + cc];
          ++cnt;
        }
      const double mean = acc / cnt;
      if (mean > best) {
        best = mean;
        bx = c;
        by = r;
      }
    }
  double lo = g[0], hi = g[0];
  for (int k = 1; k < w * h; ++k) {
    lo = g[k] < lo ? g[k] : lo;
    hi = g[k] > hi ? g[k] : hi;
  }
  const double beta0 = lo, alpha0 = hi - lo;
  const double thr = fma(alpha0, exp(-0.5), beta0);
  int M = 0;
  for (int k = 0; k < w * h; ++k) M += g[k] > thr;
  double s = sqrt(M / M_PI);
  if (s < 0.5) s = 0.5;
  out[0] = bx;
  out[1] = by;
  out[2] = out[3] = s;
  return 0;
}

int orc_peak_init_batch(const void* data, int dtype, const uint8_t* sizes,
                        const int64_t* offsets, int64_t n, double* out) {
  double g[ORC_MAXPIX];
  for (int64_t s = 0; s < n; ++s) {
    const int w = sizes[4 * s], h = sizes[4 * s + 1];
    if (w < 3 || h < 3 || w * h > ORC_MAXPIX) {
      for (int i = 0; i < 4; ++i) out[4 * s + i] = NAN;
      continue;
    }
    for (int k = 0; k < w * h; ++k)
      g[k] = dtype == 0 ? (double)((const uint16_t*)data)[offsets[s] + k]
                        : (double)((const float*)data)[offsets[s] + k];
    orc_peak_init(g, w, h, out + 4 * s);
  }
  return 0;
}
