"""Pins of the double-precision oracle against things other than itself.

Each test checks the oracle against what the paper or the mathematics fixes:
a textbook linear least-squares solve (Eqs. 3-6), finite differences
(Eqs. 7-9, 11), a generic dense solve (Eq. 14), noise-free recovery, an
explicit five-parameter fit done by scipy, brute-force grid search on tiny
spots, model special cases, and the paper's own Table 1 and Fig. 8 statistics.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize

import oracle
import spotgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid_xy(w, h):
    k = np.arange(w * h)
    return (k % w).astype(float), (k // w).astype(float)


def _profile_np(w, h, model, p):
    # the generator-independent profile used only to build inputs for the pins
    x, y = _grid_xy(w, h)
    if model == 0:
        return np.exp(-((x - p[0]) ** 2 + (y - p[1]) ** 2) / (2 * p[2] ** 2))
    return np.exp(-(x - p[0]) ** 2 / (2 * p[2] ** 2) - (y - p[1]) ** 2 / (2 * p[3] ** 2))


def _lstsq_residual(g, w, h, model, p):
    """r = h - g with (alpha, beta) from numpy's least-squares solver."""
    f = _profile_np(w, h, model, p)
    M = np.stack([f, np.ones_like(f)], 1)
    coef, *_ = np.linalg.lstsq(M, g, rcond=None)
    return M @ coef - g, coef


def _rand_spot(rng, w, h, model, noisy=True):
    n = 3 if model == 0 else 4
    p = np.array([(w - 1) / 2 + rng.uniform(-1, 1), (h - 1) / 2 + rng.uniform(-1, 1),
                  rng.uniform(1.1, 2.5), rng.uniform(1.1, 2.5)])[:n]
    if model == 0:
        p = p[:3]
    lam = rng.uniform(200, 3000) * _profile_np(w, h, model, p) + rng.uniform(10, 300)
    g = rng.poisson(lam).astype(float) if noisy else lam
    return g, p


@pytest.mark.parametrize("model", [0, 1])
def test_amplitudes_equal_linear_least_squares(model):
    """Eqs. 5-6: closed-form alpha_hat, beta_hat and chi^2 = lstsq of g on [f, 1]."""
    rng = np.random.default_rng(1)
    for trial in range(20):
        w, h = [(7, 7), (11, 9), (15, 15), (32, 32)][trial % 4]
        g, p = _rand_spot(rng, w, h, model)
        pt = p + rng.normal(0, 0.2, size=p.shape)  # away from the minimum too
        pt[2:] = np.abs(pt[2:]) + 0.5
        e = oracle.eval_spot(g, w, h, model, pt, grad=False)
        r, coef = _lstsq_residual(g, w, h, model, pt)
        assert e["rc"] == 0
        assert e["alpha"] == pytest.approx(coef[0], rel=1e-11, abs=1e-9)
        assert e["beta"] == pytest.approx(coef[1], rel=1e-11, abs=1e-9)
        assert e["chi2"] == pytest.approx(float(r @ r), rel=1e-11)


@pytest.mark.parametrize("model", [0, 1])
def test_jacobian_matches_finite_differences(model):
    """Eqs. 7-9 and 11: J = d(h - g)/dp, by central differences of the lstsq residual."""
    rng = np.random.default_rng(2)
    for trial in range(12):
        w, h = [(9, 9), (15, 15), (21, 13)][trial % 3]
        g, p = _rand_spot(rng, w, h, model)
        pt = p + rng.normal(0, 0.15, size=p.shape)
        e = oracle.eval_spot(g, w, h, model, pt, grad=True, want_J=True)
        n = len(pt)
        Jfd = np.zeros((w * h, n))
        for j in range(n):
            hstep = 1e-5 * max(1.0, abs(pt[j]))
            pp, pm = pt.copy(), pt.copy()
            pp[j] += hstep
            pm[j] -= hstep
            Jfd[:, j] = (_lstsq_residual(g, w, h, model, pp)[0] -
                         _lstsq_residual(g, w, h, model, pm)[0]) / (2 * hstep)
        scale = np.abs(Jfd).max()
        assert np.abs(e["J"] - Jfd).max() < 1e-7 * scale
        r, _ = _lstsq_residual(g, w, h, model, pt)
        # normal matrix and right-hand side from the finite-difference Jacobian
        np.testing.assert_allclose(e["A"], Jfd.T @ Jfd, rtol=1e-6, atol=1e-7 * scale ** 2)
        np.testing.assert_allclose(e["b"], -Jfd.T @ r, rtol=1e-6,
                                   atol=1e-7 * scale * np.abs(r).sum())


@pytest.mark.parametrize("model", [0, 1])
def test_gradient_is_derivative_of_chi2(model):
    """The right-hand side of Eq. 12 is -1/2 d chi^2/dp (a descent direction)."""
    rng = np.random.default_rng(3)
    for trial in range(10):
        g, p = _rand_spot(rng, 13, 13, model)
        pt = p + rng.normal(0, 0.2, size=p.shape)
        e = oracle.eval_spot(g, 13, 13, model, pt, grad=True)
        for j in range(len(pt)):
            hstep = 1e-5
            pp, pm = pt.copy(), pt.copy()
            pp[j] += hstep
            pm[j] -= hstep
            cp = oracle.eval_spot(g, 13, 13, model, pp, grad=False)["chi2"]
            cm = oracle.eval_spot(g, 13, 13, model, pm, grad=False)["chi2"]
            d = (cp - cm) / (2 * hstep)
            assert -2 * e["b"][j] == pytest.approx(d, rel=1e-6, abs=1e-6 * abs(cp))


@pytest.mark.parametrize("model", [0, 1])
def test_envelope_identity(model):
    """Sum r f = sum r = 0 at alpha_hat, beta_hat (Eq. 4), hence J^T r = alpha sum r df_j."""
    rng = np.random.default_rng(4)
    g, p = _rand_spot(rng, 15, 15, model)
    pt = p + 0.1
    e = oracle.eval_spot(g, 15, 15, model, pt, grad=True, want_J=True)
    r, coef = _lstsq_residual(g, 15, 15, model, pt)
    f = _profile_np(15, 15, model, pt)
    assert abs(r @ f) < 1e-9 * np.abs(r).sum()
    assert abs(r.sum()) < 1e-9 * np.abs(r).sum()
    # alpha * df_j is the part of J_j not in span{f, 1}; project both and compare
    Jr = e["J"].T @ r
    np.testing.assert_allclose(-e["b"], Jr, rtol=1e-10, atol=1e-10 * np.abs(Jr).max())


def test_symmetric_is_elliptical_with_equal_widths():
    """The elliptical model at sigma_x = sigma_y reduces to Eq. 10; d/dsigma = d/dsx + d/dsy."""
    rng = np.random.default_rng(5)
    g, p = _rand_spot(rng, 11, 11, 0)
    es = oracle.eval_spot(g, 11, 11, 0, p, grad=True, want_J=True)
    ee = oracle.eval_spot(g, 11, 11, 1, [p[0], p[1], p[2], p[2]], grad=True, want_J=True)
    for k in ("alpha", "beta", "chi2"):
        assert es[k] == pytest.approx(ee[k], rel=1e-13)
    np.testing.assert_allclose(es["J"][:, :2], ee["J"][:, :2], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(es["J"][:, 2], ee["J"][:, 2] + ee["J"][:, 3], rtol=1e-11,
                               atol=1e-11)


def test_damped_solve_matches_dense_solve():
    """Eq. 14: (A + lambda diag A) delta = b; a singular matrix gives NaN."""
    rng = np.random.default_rng(6)
    for n in (3, 4):
        for _ in range(20):
            X = rng.normal(size=(10, n))
            A = X.T @ X
            b = rng.normal(size=n)
            lam = 10.0 ** rng.integers(-8, 5)
            d, rc = oracle.solve(A, b, lam)
            ref = np.linalg.solve(A + lam * np.diag(np.diag(A)), b)
            assert rc == 0
            np.testing.assert_allclose(d, ref, rtol=1e-9, atol=1e-12)
    d, rc = oracle.solve(np.zeros((3, 3)), np.ones(3), 0.01)
    assert rc == 1 and np.all(np.isnan(d))


def test_pow10_is_correctly_rounded():
    for k in range(-22, 23):
        assert oracle.pow10(k) == float(f"1e{k}")


@pytest.mark.parametrize("model", [0, 1])
def test_noise_free_recovery(model):
    """Exact float64 renders are fitted back to the true parameters to 1e-9."""
    rng = np.random.default_rng(7)
    o = oracle.default_opts(max_error_per_px=0.0, max_iter=60, min_delta=0.0,
                            min_step_rel=0.0)
    for trial in range(20):
        w = h = [9, 11, 15, 21][trial % 4]
        n = 3 if model == 0 else 4
        truth = np.array([(w - 1) / 2 + rng.uniform(-1, 1), (h - 1) / 2 + rng.uniform(-1, 1),
                          rng.uniform(1.2, 2.5), rng.uniform(1.2, 2.5)])[:n]
        a, b = rng.uniform(200, 3000), rng.uniform(10, 300)
        g = a * _profile_np(w, h, model, truth) + b
        init = np.array([truth[0] + 0.4, truth[1] - 0.3, truth[2] * 1.2,
                         truth[-1] * 0.85], dtype=np.float32)
        r = oracle.fit_spot(g, w, h, model, init, o)
        got = r["params"][[0, 1, 2, 3]][:n] if model == 1 else r["params"][:3]
        assert np.abs(got - truth).max() < 1e-9, (r, truth)
        assert r["params"][4] == pytest.approx(a, rel=1e-9)
        assert r["params"][5] == pytest.approx(b, rel=1e-9, abs=1e-7)


@pytest.mark.parametrize("model", [0, 1])
def test_equals_explicit_five_parameter_fit(model):
    """Implicit amplitudes reach the minimum of the full objective of Eq. 1 (scipy LM)."""
    rng = np.random.default_rng(8)
    o = oracle.default_opts(max_error_per_px=0.0, max_iter=200, min_delta=0.0,
                            min_step_rel=1e-13)
    for trial in range(12):
        w = h = [9, 11, 15][trial % 3]
        g, p = _rand_spot(rng, w, h, model)
        init = np.concatenate([p, p[-1:]]) if model == 0 else p
        init = (init + rng.normal(0, 0.2, 4)).astype(np.float32)
        init[2:] = np.abs(init[2:]) + 0.3
        r = oracle.fit_spot(g, w, h, model, init, o)
        n = 3 if model == 0 else 4
        q0 = np.concatenate([r["params"][:n] + 0.05, [r["params"][4] * 1.1, r["params"][5] - 3]])

        def res(q):
            return q[n] * _profile_np(w, h, model, q[:n]) + q[n + 1] - g

        sol = scipy.optimize.least_squares(res, q0, method="lm", xtol=1e-15, ftol=1e-15,
                                           gtol=1e-15, max_nfev=20000)
        ref = np.concatenate([sol.x[:n], sol.x[n:]])
        got = np.concatenate([r["params"][:n], r["params"][4:6]])
        np.testing.assert_allclose(got, ref, rtol=1e-7, atol=1e-7)
        assert r["chi2"] == pytest.approx(float(sol.fun @ sol.fun), rel=1e-10)


def _grid_chi2(g, w, h, xs, ys, ss):
    """chi^2 minimised over (alpha, beta) at every (x, y, sigma) grid point."""
    px, py = _grid_xy(w, h)
    X, Y, S = np.meshgrid(xs, ys, ss, indexing="ij")
    X, Y, S = X.ravel(), Y.ravel(), S.ravel()
    best = np.full(X.shape, np.inf)
    N = w * h
    G, G2 = g.sum(), (g * g).sum()
    for c0 in range(0, X.size, 200000):
        sl = slice(c0, c0 + 200000)
        f = np.exp(-((px[None] - X[sl, None]) ** 2 + (py[None] - Y[sl, None]) ** 2) /
                   (2 * S[sl, None] ** 2))
        F, FF, FG = f.sum(1), (f * f).sum(1), f @ g
        # 2x2 normal equations solved with numpy per point, residual computed directly
        M = np.stack([np.stack([FF, F], -1), np.stack([F, np.full_like(F, N)], -1)], -2)
        rhs = np.stack([FG, np.full_like(F, G)], -1)
        coef = np.linalg.solve(M, rhs[..., None])[..., 0]
        r = coef[:, :1] * f + coef[:, 1:] - g[None]
        best[sl] = (r * r).sum(1)
    i = int(np.argmin(best))
    return best[i], (X[i], Y[i], S[i])


@pytest.mark.parametrize("side", [5, 7])
def test_global_minimum_by_grid_search(side):
    """On tiny spots the fitted chi^2 is the global minimum found by brute force."""
    rng = np.random.default_rng(9 + side)
    for trial in range(3):
        g, p = _rand_spot(rng, side, side, 0)
        init = np.array([p[0] + 0.3, p[1] - 0.2, p[2] * 1.15, 0], dtype=np.float32)
        r = oracle.fit_spot(g, side, side, 0, init,
                            oracle.default_opts(max_error_per_px=0.0, max_iter=100,
                                                min_delta=1e-14, min_step_rel=1e-12))
        # coarse grid over the whole box, then a fine grid (step 0.005) around its best
        c2, (cx, cy, cs) = _grid_chi2(g, side, side, np.arange(-0.5, side - 0.5, 0.05),
                                      np.arange(-0.5, side - 0.5, 0.05),
                                      np.arange(0.5, 4.0, 0.05))
        step = 0.005
        f2, (fx, fy, fs) = _grid_chi2(g, side, side, np.arange(cx - 0.1, cx + 0.1 + 1e-9, step),
                                      np.arange(cy - 0.1, cy + 0.1 + 1e-9, step),
                                      np.arange(cs - 0.1, cs + 0.1 + 1e-9, step))
        assert r["chi2"] <= f2 * (1 + 1e-12)
        assert abs(r["params"][0] - fx) <= step and abs(r["params"][1] - fy) <= step
        assert abs(r["params"][2] - fs) <= step


def test_degenerate_and_bad_inputs():
    o = oracle.default_opts()
    # constant spot: alpha = 0, chi^2 = 0 < N/3 -> MaxError at the first iteration
    r = oracle.fit_spot(np.full(81, 100.0), 9, 9, 0, [4, 4, 1.5, 1.5], o)
    assert r["status"] == oracle.MAX_ERROR and r["iters"] == 1 and r["chi2"] < 1e-18
    # NaN pixel -> NaN error -> NotConverged at the first iteration
    g = np.full(81, 100.0)
    g[5] = np.nan
    r = oracle.fit_spot(g, 9, 9, 0, [4, 4, 1.5, 1.5], o)
    assert r["status"] == oracle.NOT_CONVERGED and r["iters"] == 1
    # spot-level input errors
    for (w, h, model, init) in [(2, 9, 0, [1, 4, 1, 1]), (33, 32, 0, [4, 4, 1, 1]),
                                (9, 9, 7, [4, 4, 1, 1]), (9, 9, 0, [np.nan, 4, 1, 1]),
                                (9, 9, 0, [4, 4, 0.0, 1]), (9, 9, 1, [4, 4, 1.0, -1])]:
        g = np.full(w * h, 10.0)
        r = oracle.fit_spot(g, w, h, model, init, o)
        assert r["status"] == oracle.BAD_INPUT and r["iters"] == 0
        assert np.all(np.isnan(r["params"]))
    # a zero iteration budget returns the init with status MaxIter
    o0 = oracle.default_opts(max_iter=0)
    b = spotgen.config(0, n=4)
    r = oracle.fit_spot(b.spot(0).astype(float), 11, 11, 0, b.init[0], o0)
    assert r["status"] == oracle.MAX_ITER and r["iters"] == 0
    assert r["params"][0] == pytest.approx(float(b.init[0, 0]))


def test_batch_driver_matches_single_spots_and_threads():
    b = spotgen.config(3, n=300)
    r1 = oracle.fit_batch(b, threads=1)
    r4 = oracle.fit_batch(b, threads=4)
    for k in r1:
        np.testing.assert_array_equal(r1[k], r4[k])
    for s in range(0, 300, 37):
        w, h, m = (int(v) for v in b.sizes[s, :3])
        rs = oracle.fit_spot(b.spot(s).astype(float), w, h, m, b.init[s])
        np.testing.assert_array_equal(rs["params"], r1["params"][s])
        assert rs["status"] == r1["status"][s] and rs["iters"] == r1["iters"][s]


def test_table1_accuracy_statistics():
    """Table 1 (Fit2DGaussian rows) with the paper's protocol and initial values."""
    with open(os.path.join(GOLDEN, "table1_accuracy.json")) as fh:
        gold = json.load(fh)
    for row in gold["rows"]:
        b = spotgen.paper_protocol(20000, 9, row["n_signal"], row["n_background"], seed=17)
        r = oracle.fit_batch(b, threads=8)
        st = b.truth
        exy = np.concatenate([np.abs(r["params"][:, 0] - st[:, 0]),
                              np.abs(r["params"][:, 1] - st[:, 1])]) / np.tile(st[:, 2], 2)
        es = np.abs(np.abs(r["params"][:, 2]) - st[:, 2]) / st[:, 2]
        got_xy = [np.median(exy), exy.mean(), exy.std()]
        got_s = [np.median(es), es.mean(), es.std()]
        np.testing.assert_allclose(got_xy, row["xy"], rtol=0.06)
        np.testing.assert_allclose(got_s, row["sigma"], rtol=0.08)


def test_fig8_iteration_and_stop_statistics():
    """1600:40 counts: typically 4-5 iterations, MinDelta dominates, almost none exhausted."""
    with open(os.path.join(GOLDEN, "iterations_fig8.json")) as fh:
        gold = json.load(fh)["statements"]
    b = spotgen.paper_protocol(20000, 9, 1600, 40, seed=18)
    r = oracle.fit_batch(b, threads=8)
    hist = np.bincount(r["iters"], minlength=21) / b.n
    lo, hi = gold["typical_iterations"]
    assert hist[lo] + hist[hi] > 0.8
    assert int(np.argmax(hist)) in (lo, hi)
    st = np.bincount(r["status"], minlength=6) / b.n
    assert st[oracle.MIN_DELTA] > 0.5
    assert st[oracle.MAX_ITER] < 0.005
    # fewer than 1 % reach the minimal parameter change criterion (with the centre
    # measured from the ROI centre; from the corner pixel about 5 % would)
    assert st[oracle.MIN_STEP] < gold["min_step_fraction_below"]


# ---------------------------------------------------------------------------
# The loop's control flow (Levenberg-Marquardt section, Fit2DGaussian
# pseudo-code), pinned by replaying the oracle's logged trajectory with numbers
# computed here independently: chi^2 from numpy's least-squares solve of g on
# [f, 1], the normal equations from a central-difference Jacobian of that
# residual, the damped step from numpy.linalg.solve.  The replay takes each
# decision the pseudo-code prescribes and checks that the oracle took the same
# one, evaluation by evaluation, through to the returned point and status.
# ---------------------------------------------------------------------------

_DEFAULTS = dict(max_iter=20, max_error_per_px=1.0 / 3.0, min_delta=1e-6, min_step_rel=1e-4,
                 lambda0_exp10=-2, lambda_max_exp10=4, sigma_min=0.3, sigma_max_frac=1.0)


def _chi2_lstsq(g, w, h, model, p):
    r, coef = _lstsq_residual(g, w, h, model, p)
    return float(r @ r), coef


def _residual_complex(g, w, h, model, p):
    """h - g at complex shaping parameters: the 2x2 normal equations of (alpha,
    beta) solved by numpy's generic solver (analytic in p, no conjugation)."""
    x, y = _grid_xy(w, h)
    if model == 0:
        f = np.exp(-((x - p[0]) ** 2 + (y - p[1]) ** 2) / (2 * p[2] ** 2))
    else:
        f = np.exp(-(x - p[0]) ** 2 / (2 * p[2] ** 2) - (y - p[1]) ** 2 / (2 * p[3] ** 2))
    M = np.array([[np.sum(f * f), np.sum(f)], [np.sum(f), float(w * h)]])
    coef = np.linalg.solve(M, np.array([np.sum(f * g), np.sum(g)]))
    return coef[0] * f + coef[1] - g


def _normal_fd(g, w, h, model, p):
    """J^T J and J^T (g - h), J = d(h - g)/dp by complex-step differentiation of the
    residual (derivative to rounding accuracy, independent of Eqs. 7-9)."""
    n = len(p)
    J = np.zeros((w * h, n))
    for j in range(n):
        pc = p.astype(np.complex128)
        pc[j] += 1e-30j
        J[:, j] = _residual_complex(g, w, h, model, pc).imag / 1e-30
    r, _ = _lstsq_residual(g, w, h, model, p)
    return J.T @ J, -J.T @ r


def _replay(g, w, h, model, init, kw, res, events):
    """Walk the pseudo-code with independent numbers; returns the exit branch."""
    o = dict(_DEFAULTS, **kw)
    n = 3 if model == 0 else 4
    T = o["max_error_per_px"] * w * h
    smax = o["sigma_max_frac"] * max(w, h)

    def limit(q):
        q = q.copy()
        q[0] = min(max(q[0], -0.5), w - 0.5)
        q[1] = min(max(q[1], -0.5), h - 0.5)
        q[2:] = np.minimum(np.maximum(q[2:], o["sigma_min"]), smax)
        return q

    pos = 0

    def take(kind, it, k, p, d=None):
        """Check the oracle's next evaluation against the replay's; continue from the
        oracle's point (equal to the replay's up to rounding) so that rounding
        differences do not accumulate; chi^2 there by lstsq."""
        nonlocal pos
        assert pos < len(events), "the oracle stopped early"
        e = events[pos]
        pos += 1
        assert (e["kind"], e["iter"], e["k"]) == (kind, it, k), (e, kind, it, k)
        np.testing.assert_allclose(e["p"], p, rtol=1e-7, atol=1e-8)
        if d is not None:
            np.testing.assert_allclose(e["delta"], d, rtol=1e-7,
                                       atol=1e-9 * np.abs(d).max() + 1e-13)
        q = np.array(e["p"], dtype=np.float64)
        chi, _ = _chi2_lstsq(g, w, h, model, q)
        assert e["chi"] == pytest.approx(chi, rel=1e-10)
        return q, chi

    def solve(A, b, k):
        return np.linalg.solve(A + 10.0 ** k * np.diag(np.diag(A)), b)

    p = np.asarray(init, dtype=np.float32).astype(np.float64)[:n]
    # MinStep measures the centre from the centre of the ROI
    org = np.array([(w - 1) / 2.0, (h - 1) / 2.0, 0.0, 0.0])[:n]
    k, it, status, branch = o["lambda0_exp10"], 0, oracle.MAX_ITER, "max_iter"
    retried = False
    while it < o["max_iter"]:
        it += 1
        p, chi = take(oracle.EV_GRAD, it, k, p)
        A, b = _normal_fd(g, w, h, model, p)
        if chi < T:
            status, branch = oracle.MAX_ERROR, "maxerr_grad"
            break
        best = p.copy()
        d = solve(A, b, k)
        p, Chi = take(oracle.EV_TRIAL, it, k, limit(best + d), d)
        if Chi < chi:
            k -= 1
        small = bool(np.all(np.abs(d) < o["min_step_rel"] * np.abs(best - org)))
        while not small and Chi > chi and k < o["lambda_max_exp10"]:
            k += 1
            retried = True
            d = solve(A, b, k)
            p, Chi = take(oracle.EV_RETRY, it, k, limit(best + d), d)
            small = bool(np.all(np.abs(d) < o["min_step_rel"] * np.abs(best - org)))
        if Chi > chi:
            p = best
            status = oracle.NOT_CONVERGED
            branch = "cap" if (not small and k >= o["lambda_max_exp10"]) else "nc_small_step"
            break
        if Chi < T:
            status, branch = oracle.MAX_ERROR, "maxerr_trial"
            break
        if chi * (1 - o["min_delta"]) < Chi:
            status, branch = oracle.MIN_DELTA, "min_delta"
            break
        if small:
            status, branch = oracle.MIN_STEP, "min_step"
            break
    assert pos == len(events), "the oracle evaluated more than the pseudo-code prescribes"
    assert (res["status"], res["iters"]) == (status, it)
    np.testing.assert_allclose(res["params"][:n] if model else res["params"][:3], p,
                               rtol=1e-7, atol=1e-8)
    chi_end, coef = _chi2_lstsq(g, w, h, model, p)
    assert res["chi2"] == pytest.approx(chi_end, rel=1e-9)
    np.testing.assert_allclose(res["params"][4:6], coef, rtol=1e-8, atol=1e-8)
    return branch + ("+retry" if retried and branch != "cap" else "")


def _replay_cases():
    """(batch, option overrides, spots per exit branch) with every exit of the loop."""
    return [
        (spotgen.workload("mixed_low_contrast", n=2500), dict(lambda0_exp10=-8,
                                                             lambda_max_exp10=-5), 12),
        (spotgen.paper_protocol(1500, 4, 400, 40), dict(lambda_max_exp10=-2), 12),
        (spotgen.paper_protocol(1500, 4, 400, 40), dict(), 8),
        (spotgen.config(0, n=400), dict(max_error_per_px=230.0), 8),
        (spotgen.noise_free(120), dict(), 6),
        (spotgen.config(1, n=300), dict(), 6),
        (spotgen.paper_protocol(800, 7, 160, 49), dict(), 6),
    ]


def _replay_batch(batch, kw, per_branch, fit=None):
    fit = fit or oracle.fit_spot_traced
    o = oracle.default_opts(**kw)
    seen = {}
    for s in range(batch.n):
        w, h, m = (int(v) for v in batch.sizes[s, :3])
        g = batch.spot(s).astype(np.float64).ravel()
        res, ev = fit(g, w, h, m, batch.init[s], o)
        # decisions closer to their threshold than the two sides' rounding can
        # resolve are left out
        if res["margin_chi"] < 1e-9 or res["margin_step"] < 1e-6:
            continue
        key = res["status"], len(ev) > 0 and ev[-1]["kind"], \
            any(e["kind"] == oracle.EV_RETRY for e in ev)
        if seen.get(key, 0) >= per_branch:
            continue
        seen[key] = seen.get(key, 0) + 1
        yield _replay(g, w, h, m, batch.init[s], kw, res, ev)


def test_loop_trajectory_replays_the_pseudo_code():
    """Every exit of the loop, each reached by the oracle on these inputs: the
    damping cap with the best point restored (NotConverged), MaxError before and
    after a trial, MinDelta and MinStep with and without retries, and an
    exhausted iteration budget."""
    branches = {}
    for batch, kw, per in _replay_cases():
        for br in _replay_batch(batch, kw, per):
            branches[br] = branches.get(br, 0) + 1
    print(branches)
    for want in ("cap", "maxerr_grad", "maxerr_trial", "min_delta", "min_delta+retry",
                 "min_step", "max_iter"):
        assert branches.get(want, 0) > 0, (want, branches)


def test_no_retry_when_the_cap_is_the_start_damping():
    """lambda_max = lambda0: a first trial that is worse ends the fit at iteration 1
    with NotConverged and the start point, with no retry (checked against chi^2
    computed here)."""
    b = spotgen.paper_protocol(600, 4, 400, 40)
    o = oracle.default_opts(lambda_max_exp10=-2)
    hits = 0
    for s in range(b.n):
        g = b.spot(s).astype(np.float64).ravel()
        p0 = b.init[s].astype(np.float64)[:3]
        chi0, _ = _chi2_lstsq(g, 4, 4, 0, p0)
        A, bv = _normal_fd(g, 4, 4, 0, p0)
        d = np.linalg.solve(A + 1e-2 * np.diag(np.diag(A)), bv)
        p1 = p0 + d
        p1[:2] = np.clip(p1[:2], -0.5, 3.5)
        p1[2] = np.clip(p1[2], 0.3, 4.0)
        chi1, _ = _chi2_lstsq(g, 4, 4, 0, p1)
        if not chi1 > chi0 * (1 + 1e-9):
            continue
        hits += 1
        r = oracle.fit_spot(g, 4, 4, 0, b.init[s], o)
        assert r["status"] == oracle.NOT_CONVERGED and r["iters"] == 1
        assert r["n_trial"] == 1
        np.testing.assert_array_equal(r["params"][:3], p0)
    assert hits >= 10


_MISTAKES = {
    # one retry too many: the damping may exceed the cap
    "retry_past_cap": ("k < o->lambda_max_exp10", "k <= o->lambda_max_exp10"),
    # NotConverged without restoring the best point
    "no_restore": ("memcpy(p, best, sizeof(double) * n);\n      status = ORC_NOT_CONVERGED;",
                   "status = ORC_NOT_CONVERGED;"),
    # MaxError tested on the error before the step instead of the trial's
    "maxerr_on_chi": ("if (chi_below(Chi, T, T, mc)) { status = ORC_MAX_ERROR; break; }",
                      "if (chi_below(chi, T, T, mc)) { status = ORC_MAX_ERROR; break; }"),
    # the damping not reduced after an improving first trial
    "no_decrease": ("if (chi_below(Chi, chi * (1.0 - tau), chi, mc)) --k;",
                    "if (chi_below(Chi, chi * (1.0 - tau), chi, mc)) k = k;"),
}


@pytest.mark.parametrize("mistake", list(_MISTAKES))
def test_replay_catches_planted_loop_mistakes(tmp_path, mistake):
    """A copy of the oracle with one control-flow mistake planted fails the replay."""
    import ctypes
    import subprocess
    src = open(oracle.SRC_PATH).read()
    old, new = _MISTAKES[mistake]
    assert src.count(old) >= 1, mistake
    c = tmp_path / "mutant.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=gnu99", "-ffp-contract=off",
                    "-I", os.path.dirname(oracle.SRC_PATH), "-o", str(so), str(c), "-lm",
                    "-lpthread"], check=True)
    mutant = oracle.bind(ctypes.CDLL(str(so)))
    saved = oracle._lib
    oracle._lib = mutant
    try:
        caught = False
        for batch, kw, per in _replay_cases():
            try:
                for _ in _replay_batch(batch, kw, per):
                    pass
            except AssertionError:
                caught = True
                break
        assert caught, f"planted mistake {mistake} passed the replay"
    finally:
        oracle._lib = saved


# ---------------------------------------------------------------------------
# Start values (centroid / second moments): outside the paper's method, pinned
# by hand-built images whose estimate is known exactly.
# ---------------------------------------------------------------------------
def test_moment_init_single_bright_pixel():
    g = np.full((9, 11), 100.0)
    g[4, 3] = 500.0
    out = oracle.moment_init(g, 11, 9, 0)
    np.testing.assert_array_equal(out, [3.0, 4.0, 0.8, 0.8])  # zero spread, clamped to 0.8


def test_moment_init_flat_image_falls_back_to_roi_centre():
    out = oracle.moment_init(np.full((7, 9), 42.0), 9, 7, 1)
    np.testing.assert_array_equal(out, [4.0, 3.0, 1.5, 1.5])


def test_moment_init_known_moments():
    # background 50 everywhere; +100 at (x +- 3, y) and (x, y +- 1) around (5, 5):
    # centroid (5, 5), var_x = 2*9*100/400 = 4.5, var_y = 2*1*100/400 = 0.5
    g = np.full((11, 11), 50.0)
    for (r, c) in [(5, 2), (5, 8), (4, 5), (6, 5)]:
        g[r, c] = 150.0
    sym = oracle.moment_init(g, 11, 11, 0)
    ell = oracle.moment_init(g, 11, 11, 1)
    np.testing.assert_allclose(sym, [5.0, 5.0, np.sqrt(2.5), np.sqrt(2.5)], rtol=1e-15)
    np.testing.assert_allclose(ell, [5.0, 5.0, np.sqrt(4.5), 0.8], rtol=1e-15)  # sigma_y clamped


def test_moment_init_ring_median_is_mean_of_middle_values():
    # 9x9 ring of 32 pixels: 16 at 10 and 16 at 20, the 20s placed symmetrically
    # (odd columns of the top and bottom rows, odd rows of the side columns), so
    # b0 = 15 and the ring's own weights (5 each) centre on (4, 4).  Interior 0
    # except 25 at (x=3, y=4) and 45 at (x=5, y=4): weights 10 and 30, so
    # cx = (80*4 + 10*3 + 30*5) / 120; b0 = 10 or 20 would give 860/210 or 140/30
    w = h = 9
    g = np.zeros((h, w))
    for c in range(w):
        g[0, c] = g[h - 1, c] = 20.0 if c % 2 else 10.0
    for r in range(1, h - 1):
        g[r, 0] = g[r, w - 1] = 20.0 if r % 2 else 10.0
    g[4, 3] = 25.0
    g[4, 5] = 45.0
    out = oracle.moment_init(g, w, h, 0)
    assert out[0] == pytest.approx(500.0 / 120.0, rel=1e-15) and out[1] == 4.0


def test_moment_init_matches_the_vectorised_estimate():
    # an independent (numpy, vectorised) implementation of the same estimate
    for name in ("small_11x11", "mixed_7to32", "precision_32x32_ell"):
        b = spotgen.workload(name, n=600)
        mine = oracle.moment_init_batch(b)
        for s in range(0, b.n, 7):
            w, h, model = int(b.sizes[s, 0]), int(b.sizes[s, 1]), int(b.sizes[s, 2])
            img = b.spot(s).reshape(1, h, w).astype(np.float64)
            ref = spotgen.moment_init(img, model)[0]
            np.testing.assert_allclose(mine[s], ref, rtol=1e-12, atol=1e-12)


def test_moment_init_rejects_unusable_shapes():
    assert np.all(np.isnan(oracle.moment_init(np.ones(6), 2, 3, 0)))
    assert np.all(np.isnan(oracle.moment_init(np.ones(25), 5, 5, 7)))


# ---------------------------------------------------------------------------
# The paper's start values (Results section): 3x3 moving average, brightest
# smoothed pixel, sigma = sqrt(M / pi).  Pinned by images whose smoothed
# maximum and above-threshold count are known by hand, and by a library 2-D
# convolution with numpy's first-occurrence argmax.
# ---------------------------------------------------------------------------
def test_peak_init_lone_bright_pixel():
    s1 = math.sqrt(1.0 / math.pi)
    g = np.full((9, 11), 100.0)
    g[4, 5] = 1000.0
    # every full window holding the bright pixel has mean 200: nine ties, the
    # first in row-major order is the window centred one up and one left
    np.testing.assert_array_equal(oracle.peak_init(g, 11, 9), [4.0, 3.0, s1, s1])
    g = np.full((9, 11), 100.0)
    g[0, 5] = 1000.0
    # on the top edge the windows hold six pixels: mean 250 beats the full ones' 200
    np.testing.assert_array_equal(oracle.peak_init(g, 11, 9), [4.0, 0.0, s1, s1])
    g = np.full((9, 11), 100.0)
    g[8, 10] = 1000.0
    # in a corner the window holds four pixels: mean 325
    np.testing.assert_array_equal(oracle.peak_init(g, 11, 9), [10.0, 8.0, s1, s1])


def test_peak_init_flat_image():
    # no pixel exceeds the threshold (= the flat value): M = 0, sigma floored at 0.5
    np.testing.assert_array_equal(oracle.peak_init(np.full((7, 9), 42.0), 9, 7),
                                  [0.0, 0.0, 0.5, 0.5])


def test_peak_init_plateaus_of_known_area():
    g = np.full((9, 13), 100.0)
    g[3:6, 5:8] = 500.0  # 3x3 block centred on (x=6, y=4): its centre alone averages 500
    np.testing.assert_array_equal(oracle.peak_init(g, 13, 9),
                                  [6.0, 4.0, 3.0 / math.sqrt(math.pi), 3.0 / math.sqrt(math.pi)])
    g = np.full((9, 13), 100.0)
    g[2:4, 7:9] = 500.0  # 2x2 block: its four pixels tie, the first is its top-left corner
    np.testing.assert_array_equal(oracle.peak_init(g, 13, 9),
                                  [7.0, 2.0, 2.0 / math.sqrt(math.pi), 2.0 / math.sqrt(math.pi)])


def test_peak_init_threshold():
    # min 0, max 1000: threshold 1000 exp(-1/2) = 606.53...; 607 counts, 606 does not
    g = np.zeros((8, 8))
    g[0, 0] = 1000.0
    g[5, 1:4] = 607.0
    g[6, 1:6] = 606.0
    out = oracle.peak_init(g, 8, 8)
    assert out[2] == math.sqrt(4.0 / math.pi)


def test_peak_init_matches_library_convolution():
    from scipy.signal import convolve2d
    k = np.ones((3, 3))
    for S, sig, bg in ((4, 400, 40), (9, 400, 40), (11, 1600, 0), (21, 1000, 441)):
        b = spotgen.paper_protocol(300, S, sig, bg, seed=5)
        mine = oracle.peak_init_batch(b)
        for s in range(b.n):
            img = b.spot(s).reshape(S, S).astype(np.float64)
            sm = convolve2d(img, k, mode="same") / convolve2d(np.ones_like(img), k, mode="same")
            y0, x0 = np.divmod(int(np.argmax(sm)), S)
            lo, hi = img.min(), img.max()
            M = int((img > (hi - lo) * math.exp(-0.5) + lo).sum())
            sg = max(math.sqrt(M / math.pi), 0.5)
            np.testing.assert_array_equal(mine[s], [x0, y0, sg, sg])


def test_peak_init_matches_the_generator_recipe():
    # the generator's vectorised version of the same recipe (the start values of
    # the paper-protocol batches), an independent implementation
    for S in (5, 9, 16, 32):
        b = spotgen.paper_protocol(500, S, 400, 40, seed=6)
        np.testing.assert_array_equal(oracle.peak_init_batch(b).astype(np.float32), b.init)


def test_peak_init_rejects_unusable_shapes():
    assert np.all(np.isnan(oracle.peak_init(np.ones(6), 2, 3)))
    assert np.all(np.isnan(oracle.peak_init(np.ones(33 * 32), 33, 32)))


# ---------------------------------------------------------------------------
# Drift tracking of fiducial markers (averaging positions over markers and
# frames, Introduction): pinned by exact shifts, excluded markers and a linear
# drift whose window means are known in closed form.
# ---------------------------------------------------------------------------
def _marker_frames(F, M, shift):
    ref = np.stack([np.arange(M) * 0.5 + 3.0, np.arange(M) * 0.25 + 4.0], axis=1)
    p = np.zeros((F, M, 6))
    for f in range(F):
        p[f, :, 0] = ref[:, 0] + shift[f][0]
        p[f, :, 1] = ref[:, 1] + shift[f][1]
    return p, np.full((F, M), oracle.MIN_DELTA), ref


def test_drift_exact_shift_and_excluded_markers():
    p, st, ref = _marker_frames(3, 10, [(0.25, -0.5)] * 3)
    # markers whose fit did not stop on a convergence test do not count
    st[1, 3] = oracle.NOT_CONVERGED
    p[1, 3, 0] += 5.0
    st[1, 4] = oracle.MAX_ITER
    p[1, 4, 1] -= 7.0
    st[2, :] = oracle.BAD_INPUT  # a frame with no usable marker
    out = oracle.drift_track(p, st, ref, window=8)
    np.testing.assert_array_equal(out[0], [0.25, -0.5, 0.25, -0.5, 10, 1])
    np.testing.assert_array_equal(out[1], [0.25, -0.5, 0.25, -0.5, 8, 2])
    assert np.all(np.isnan(out[2, :2])) and out[2, 4] == 0
    np.testing.assert_array_equal(out[2, 2:4], [0.25, -0.5])  # the window keeps the others
    assert out[2, 5] == 2


def test_drift_window_mean_of_linear_drift():
    F, W = 12, 4
    p, st, ref = _marker_frames(F, 6, [(0.125 * f, -0.0625 * f) for f in range(F)])
    out = oracle.drift_track(p, st, ref, window=W)
    for f in range(F):
        k = min(W, f + 1)
        mean_f = f - (k - 1) / 2.0  # mean of f-k+1 .. f
        assert out[f, 2] == pytest.approx(0.125 * mean_f, abs=1e-15)
        assert out[f, 3] == pytest.approx(-0.0625 * mean_f, abs=1e-15)
        assert out[f, 5] == k
