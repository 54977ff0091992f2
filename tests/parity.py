"""Comparison of GPU fit results with the double-precision oracle.

Tolerances (per spot): |dx|, |dy| < 1e-3 px; relative sigma, alpha, beta < 1e-4;
relative chi^2 < 1e-5; identical status and iteration count.  A spot whose
oracle trajectory passes a decision closer than the kernel's chi^2 error to its
threshold ("knife-edge": the oracle logs the smallest relative margin of every
chi^2 comparison and every step-size comparison it makes) may legitimately take
the other branch; so may a spot whose trajectory passes an ill-conditioned
damped solve (the oracle logs the smallest ratio of a Cholesky pivot to its
diagonal entry: below pivot_band, rounding in the normal equations moves the
step by more than the decisions can absorb).  Such spots are counted and
reported, and must still satisfy the parameter tolerances when they end with
the same status and are not ill-conditioned.

Degenerate fits (with sigma_min given): an oracle fit that ends with a
non-positive amplitude (no spot above the background) or with a width on the
lower bound of limit() (a profile narrower than a pixel, whose position and
amplitude trade off along the nearest pixel's value) has no unique minimum at
the stopping resolution of the loop: both sides may stop anywhere along the flat
direction, and a trajectory that wanders along such a direction for several
iterations can end after a different number of them, or at a different point,
on the other side's rounding.  Such spots (counted as n_degenerate) are excused
from the status, iteration and parameter comparison and must instead end valid:
a stop reason other than BAD_INPUT, finite parameters, widths not below the
bound.  Callers bound how many there may be.
"""
from __future__ import annotations

import numpy as np

TOL_XY = 1e-3
TOL_REL = 1e-4
TOL_CHI = 1e-5


def _rel(a, b):
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.abs(a / b - 1.0)


def compare(g: dict, r: dict, chi_band: float, step_band: float, model=None,
            pivot_band: float = 0.0, sigma_min=None) -> dict:
    """g: GPU outputs (params [n,6] f32, chi2, iters, status); r: oracle.fit_batch dict."""
    gp = np.asarray(g["params"], dtype=np.float64)
    rp = r["params"]
    n = len(rp)
    bad_in = r["status"] == 5
    both_nan = np.isnan(gp) & np.isnan(rp)
    dxy = np.where(both_nan[:, :2], 0.0, np.abs(gp[:, :2] - rp[:, :2])).max(1)
    # widths relative to themselves; amplitude and background relative to the
    # spot's level, so that a degenerate spot (alpha = 0, or beta ~ 0) compares sanely
    level = np.maximum(np.abs(rp[:, 4]), np.abs(rp[:, 5]))
    rel_s = _rel(gp[:, 2:4], rp[:, 2:4])
    rel_a = np.abs(gp[:, 4] - rp[:, 4]) / np.maximum(np.abs(rp[:, 4]), 1e-3 * level)
    rel_b = np.abs(gp[:, 5] - rp[:, 5]) / np.maximum(np.abs(rp[:, 5]), 1e-3 * level)
    rel = np.concatenate([rel_s, rel_a[:, None], rel_b[:, None]], 1)
    rel = np.where(both_nan[:, 2:6], 0.0, rel)
    relmax = rel.max(1)
    gc = np.asarray(g["chi2"], np.float64)
    rchi = np.abs(gc - r["chi2"]) / np.maximum(np.abs(r["chi2"]), 1e-6)
    rchi = np.where(np.isnan(gc) & np.isnan(r["chi2"]), 0.0, rchi)
    same_status = g["status"] == r["status"]
    same_iters = g["iters"] == r["iters"]
    knife = (r["margin_chi"] < chi_band) | (r["margin_step"] < step_band)
    ill = r["min_pivot"] < pivot_band if "min_pivot" in r else np.zeros(n, bool)
    knife = knife | ill
    in_tol = (dxy < TOL_XY) & (relmax < TOL_REL) & (rchi < TOL_CHI)
    deg = np.zeros(n, bool)
    if sigma_min is not None:
        deg = ~bad_in & ((rp[:, 4] <= 0.0) |
                         (np.minimum(rp[:, 2], rp[:, 3]) <= sigma_min * (1.0 + 1e-9)))
        valid = np.all(np.isfinite(gp), 1) & (g["status"] != 5) & \
            (np.minimum(gp[:, 2], gp[:, 3]) >= sigma_min * (1.0 - 1e-6))
        in_tol = np.where(deg, valid, in_tol)
    in_tol = np.where(bad_in, True, in_tol)
    # BAD_INPUT: status must match and outputs must be NaN on both sides
    nan_ok = np.all(np.isnan(gp[bad_in]))
    same = same_status & same_iters
    knife = knife | deg
    strict = ~knife
    return dict(
        n=n,
        n_knife=int(knife.sum()),
        status_mismatch=int((~same_status).sum()),
        iters_mismatch=int((~same_iters).sum()),
        strict_mismatch=int((strict & ~same).sum()),
        tol_fail_same=int((same & ~in_tol).sum()),
        tol_fail_any=int((~in_tol).sum()),
        tol_fail_strict=int((~knife & ~in_tol).sum()),
        n_ill=int(ill.sum()),
        n_degenerate=int(deg.sum()),
        max_dxy=float(np.nanmax(np.where(bad_in, 0, dxy))) if n else 0.0,
        max_rel=float(np.nanmax(np.where(bad_in, 0, relmax))) if n else 0.0,
        max_rchi=float(np.nanmax(np.where(bad_in, 0, rchi))) if n else 0.0,
        med_rchi=float(np.nanmedian(rchi[~bad_in])) if (~bad_in).any() else 0.0,
        bad_input_nan=bool(nan_ok),
        strict_mask=strict,
        mismatch_idx=np.nonzero(~same)[0],
        fail_idx=np.nonzero((strict & ~same) | (~knife & ~in_tol))[0],
    )


def describe(g: dict, r: dict, idx, limit: int = 8) -> str:
    """Both sides' results for the listed spots (for failure messages)."""
    lines = []
    for s in list(idx)[:limit]:
        lines.append(
            f"spot {s}: gpu status {int(g['status'][s])} iters {int(g['iters'][s])} "
            f"params {np.round(np.asarray(g['params'][s], np.float64), 6).tolist()} | oracle "
            f"status {int(r['status'][s])} iters {int(r['iters'][s])} "
            f"params {np.round(r['params'][s], 6).tolist()} margins chi "
            f"{r['margin_chi'][s]:.2e} step {r['margin_step'][s]:.2e} pivot "
            f"{r.get('min_pivot', np.ones(len(r['status'])))[s]:.2e}")
    return "\n".join(lines)


def summary(name: str, c: dict) -> str:
    return (f"{name}: n={c['n']} knife={c['n_knife']} (ill-conditioned {c['n_ill']}) "
            f"degenerate={c.get('n_degenerate', 0)} "
            f"status_mis={c['status_mismatch']} "
            f"iters_mis={c['iters_mismatch']} strict_mis={c['strict_mismatch']} "
            f"tol_fail(same)={c['tol_fail_same']} tol_fail(any)={c['tol_fail_any']} "
            f"max|dxy|={c['max_dxy']:.2e} max_rel={c['max_rel']:.2e} "
            f"max_rchi={c['max_rchi']:.2e} med_rchi={c['med_rchi']:.2e}")
