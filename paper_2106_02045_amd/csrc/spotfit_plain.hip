// spotfit_plain.hip -- the paper's own mapping, kept as the baseline the batched
// kernels are measured against (Implementation section of Leutenegger & Weber):
// one thread per pixel, one workgroup per spot (an integer number of
// wavefronts, at most 1024 pixels), every quantity summed by its own Sum()
// call (a wavefront reduction plus a shared-memory combine across wavefronts),
// and single precision throughout: parameters, amplitudes, sums, the 3x3 / 4x4
// step and the stop tests.  The Levenberg-Marquardt loop is the Fit2DGaussian
// pseudo-code with the same readings as the other kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spotfit.h"
#include "spotfit_internal.h"
#include "xlane.h"

namespace sf {
namespace plain {

constexpr int kMaxWaves = 16;  // 1024 threads

// Sum of v over the workgroup, returned to every thread (one value per call,
// as the paper's Sum).
__device__ __forceinline__ float block_sum(float v, float* sh, int nw) {
  float t = v;
  finish<0>(t);  // wavefront total on every lane
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[wave] = t;
  __syncthreads();
  float s = 0.f;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}

template <int NP>
__device__ __forceinline__ void solve_f(const float (&A)[NP][NP], const float (&b)[NP], float lam,
                                        float (&d)[NP]) {
  float L[NP][NP];
  float y[NP];
  bool ok = true;
  for (int j = 0; j < NP; ++j) {
    float s = A[j][j] + lam * A[j][j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    ok = ok && s > 0.f;
    L[j][j] = __builtin_sqrtf(s);
    for (int i = j + 1; i < NP; ++i) {
      float t = A[i][j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  for (int i = 0; i < NP; ++i) {
    float t = b[i];
    for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
    y[i] = t / L[i][i];
  }
  for (int i = NP - 1; i >= 0; --i) {
    float t = y[i];
    for (int k = i + 1; k < NP; ++k) t -= L[k][i] * d[k];
    d[i] = t / L[i][i];
  }
  for (int i = 0; i < NP; ++i) ok = ok && __builtin_isfinite(d[i]);
  if (!ok)
    for (int i = 0; i < NP; ++i) d[i] = __builtin_nanf("");
}

__device__ __forceinline__ float pow10f_i(int k) {
  float t = 1.f;
  const int m = k < 0 ? -k : k;
  for (int i = 0; i < m; ++i) t *= 10.f;
  return k < 0 ? 1.f / t : t;
}

__device__ __forceinline__ float clampf_n(float v, float lo, float hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

struct Pix {
  float g, x, y, m;  // value, column, row, 1 inside the spot / 0 on idle threads
};

// Gaussian2D: model at p; with grad also the normal equations.  Returns chi^2.
template <int MODEL>
__device__ float gauss2d(const Pix& px, const float* p, int N, float G, float* sh, int nw,
                         bool grad, float& a, float& b, float (*A)[4], float* bv) {
  constexpr int NP = MODEL == SPOTFIT_SYM ? 3 : 4;
  const float sx = p[2], sy = MODEL == SPOTFIT_SYM ? p[2] : p[3];
  const float isx2 = 1.f / (sx * sx), isy2 = 1.f / (sy * sy);
  const float dx = px.x - p[0], dy = px.y - p[1];
  const float q = dx * dx * isx2 + dy * dy * isy2;
  const float f = px.m * __builtin_amdgcn_exp2f(q * -0.72134752f);  // exp(-q/2)
  // AlphaBeta (Eq. 6)
  const float F = block_sum(f, sh, nw);
  const float FF = block_sum(f * f, sh, nw);
  const float FG = block_sum(f * px.g, sh, nw);
  const float Nf = float(N);
  const float D = Nf * FF - F * F;
  a = (Nf * FG - F * G) / D;
  b = (G * FF - F * FG) / D;
  const float r = px.m * (a * f + b - px.g);
  float chi = block_sum(r * r, sh, nw);
  if (!(D > 0.f) || !__builtin_isfinite(chi)) chi = __builtin_nanf("");
  if (!grad) return chi;
  // Eq. 11 and its elliptical analogue
  float df[NP];
  df[0] = dx * isx2 * f;
  df[1] = dy * isy2 * f;
  if constexpr (MODEL == SPOTFIT_SYM) {
    df[2] = (dx * dx + dy * dy) * isx2 / sx * f;
  } else {
    df[2] = dx * dx * isx2 / sx * f;
    df[3] = dy * dy * isy2 / sy * f;
  }
  float da[NP], db[NP];
  for (int j = 0; j < NP; ++j) {  // Eqs. 7-8, one Sum per quantity
    const float dF = block_sum(df[j], sh, nw);
    const float dFF = 2.f * block_sum(f * df[j], sh, nw);
    const float dFG = block_sum(px.g * df[j], sh, nw);
    const float gam = Nf * dFF - 2.f * F * dF;
    da[j] = (Nf * dFG - G * dF - a * gam) / D;
    db[j] = (G * dFF - FG * dF - F * dFG - b * gam) / D;
  }
  float J[NP];
  for (int j = 0; j < NP; ++j) J[j] = px.m * (da[j] * f + a * df[j] + db[j]);  // Eq. 9
  for (int i = 0; i < NP; ++i) {
    bv[i] = -block_sum(J[i] * r, sh, nw);
    for (int j = i; j < NP; ++j) {
      A[i][j] = block_sum(J[i] * J[j], sh, nw);
      A[j][i] = A[i][j];
    }
  }
  return chi;
}

template <int MODEL>
__device__ void fit(const Pix& px, int N, int w, int h, float G, const float* init, float* sh,
                    int nw, const KOpts& o, float* out6, float& chi_res, int& it_out,
                    int& status_out, int& ng_out, int& nt_out) {
  constexpr int NP = MODEL == SPOTFIT_SYM ? 3 : 4;
  float p[4] = {init[0], init[1], init[2], MODEL == SPOTFIT_SYM ? init[2] : init[3]};
  float best[4], delta[NP];
  float A[4][4], bv[4];
  float a, b, ta, tb;
  const float T = float(o.max_error_per_px) * float(N);
  const float tau = float(o.tie_tau);
  const float smax = float(o.sigma_max_frac) * float(w > h ? w : h);
  int k = o.lambda0_exp10, it = 0, status = SPOTFIT_MAX_ITER, ng = 0, nt = 0;
  float chi = 0.f;
  (void)tb;
  auto limit = [&](float* q) {
    q[0] = clampf_n(q[0], -0.5f, float(w) - 0.5f);
    q[1] = clampf_n(q[1], -0.5f, float(h) - 0.5f);
    q[2] = clampf_n(q[2], float(o.sigma_min), smax);
    if (MODEL == SPOTFIT_ELL) q[3] = clampf_n(q[3], float(o.sigma_min), smax);
  };
  auto small_all = [&]() {
    bool s = true;
    // the centre coordinates measured from the centre of the ROI
    const float org[2] = {0.5f * float(w - 1), 0.5f * float(h - 1)};
    for (int j = 0; j < NP; ++j)
      s = s && fabsf(delta[j]) < float(o.min_step_rel) * fabsf(best[j] - (j < 2 ? org[j] : 0.f));
    return s;
  };
  float chi_out = 0.f;  // error at the point that is returned
  // the error at the start point, needed only with a zero iteration budget
  if (o.max_iter <= 0) chi_out = gauss2d<MODEL>(px, p, N, G, sh, nw, false, a, b, A, bv);
  while (it < o.max_iter) {
    ++it;
    ++ng;
    chi = gauss2d<MODEL>(px, p, N, G, sh, nw, true, a, b, A, bv);
    chi_out = chi;
    if (__builtin_isnan(chi)) { status = SPOTFIT_NOT_CONVERGED; break; }
    if (chi < T) { status = SPOTFIT_MAX_ERROR; break; }
    for (int j = 0; j < 4; ++j) best[j] = p[j];
    const float ba = a, bb = b;
    float Am[NP][NP], b2[NP];
    for (int i = 0; i < NP; ++i) {
      b2[i] = bv[i];
      for (int j = 0; j < NP; ++j) Am[i][j] = A[i][j];
    }
    solve_f<NP>(Am, b2, pow10f_i(k), delta);
    for (int j = 0; j < NP; ++j) p[j] = best[j] + delta[j];
    limit(p);
    float Chi = gauss2d<MODEL>(px, p, N, G, sh, nw, false, ta, tb, A, bv);
    ++nt;
    if (Chi < chi * (1.f - tau)) --k;
    while (!small_all() && chi * (1.f + tau) < Chi && k < o.lambda_max_exp10) {
      ++k;
      solve_f<NP>(Am, b2, pow10f_i(k), delta);
      for (int j = 0; j < NP; ++j) p[j] = best[j] + delta[j];
      limit(p);
      Chi = gauss2d<MODEL>(px, p, N, G, sh, nw, false, ta, tb, A, bv);
      ++nt;
    }
    if (chi * (1.f + tau) < Chi || __builtin_isnan(Chi)) {
      for (int j = 0; j < 4; ++j) p[j] = best[j];
      a = ba;
      b = bb;
      status = SPOTFIT_NOT_CONVERGED;
      break;
    }
    a = ta;
    b = tb;
    chi_out = Chi;
    if (Chi < T) { status = SPOTFIT_MAX_ERROR; break; }
    if (chi * (1.f - float(o.min_delta)) < Chi) { status = SPOTFIT_MIN_DELTA; break; }
    if (small_all()) { status = SPOTFIT_MIN_STEP; break; }
  }
  out6[0] = p[0];
  out6[1] = p[1];
  out6[2] = p[2];
  out6[3] = MODEL == SPOTFIT_SYM ? p[2] : p[3];
  out6[4] = a;
  out6[5] = b;
  chi_res = chi_out;
  it_out = it;
  status_out = status;
  ng_out = ng;
  nt_out = nt;
}

__global__ __launch_bounds__(1024) void fit_plain_kernel(KArgs ka) {
  __shared__ float sh[kMaxWaves];
  const int64_t s = blockIdx.x;
  const spotfit_shape_t shp = ka.sizes[s];
  const int w = shp.w, h = shp.h, model = shp.model, N = w * h;
  const float* in = ka.init + 4 * s;
  const bool ell = model == SPOTFIT_ELL;
  const bool bad = w < 3 || h < 3 || N > ka.opt.max_pixels || w > ka.opt.max_side ||
                   h > ka.opt.max_side || N > int(blockDim.x) ||
                   (model != SPOTFIT_SYM && !ell) || !__builtin_isfinite(in[0]) ||
                   !__builtin_isfinite(in[1]) || !__builtin_isfinite(in[2]) || !(in[2] > 0.f) ||
                   (ell && (!__builtin_isfinite(in[3]) || !(in[3] > 0.f)));
  float out6[6];
  float chi = 0.f;
  int it = 0, status = SPOTFIT_BAD_INPUT, ng = 0, nt = 0;
  if (bad) {
    for (int q = 0; q < 6; ++q) out6[q] = __builtin_nanf("");
    chi = __builtin_nanf("");
  } else {
    const int k = threadIdx.x;
    const int nw = (N + 63) >> 6;  // wavefronts that hold pixels
    Pix px;
    px.m = k < N ? 1.f : 0.f;
    px.g = 0.f;
    if (k < N)
      px.g = ka.dtype == SPOTFIT_U16
                 ? float(static_cast<const uint16_t*>(ka.data)[ka.offsets[s] + k])
                 : static_cast<const float*>(ka.data)[ka.offsets[s] + k];
    px.x = float(k % w);
    px.y = float(k / w);
    const float G = block_sum(px.g, sh, nw);
    if (ell)
      fit<SPOTFIT_ELL>(px, N, w, h, G, in, sh, nw, ka.opt, out6, chi, it, status, ng, nt);
    else
      fit<SPOTFIT_SYM>(px, N, w, h, G, in, sh, nw, ka.opt, out6, chi, it, status, ng, nt);
  }
  if (threadIdx.x == 0) {
    for (int q = 0; q < 6; ++q) ka.params_out[6 * s + q] = out6[q];
    ka.chi2_out[s] = chi;
    ka.iters_out[s] = it;
    ka.status_out[s] = status;
    if (ka.evals_out) {
      ka.evals_out[2 * s] = ng;
      ka.evals_out[2 * s + 1] = nt;
    }
  }
}

}  // namespace plain

// One workgroup per spot, threads = the wavefronts needed for max_pixels.
hipError_t launch_plain_kernel(const KArgs& ka, int threads, hipStream_t st) {
  hipLaunchKernelGGL(plain::fit_plain_kernel, dim3((unsigned)ka.n), dim3(threads), 0, st, ka);
  return hipGetLastError();
}

}  // namespace sf
