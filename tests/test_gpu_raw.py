"""Raw spots in, fits out in one launch (spotfit_fit_raw), against the
composition it replaces: the start values it reports against the oracle's
centroid / second-moment estimate (and against spotfit_moment_init bit for bit
where the lane groups match), the fit against spotfit_fit_spots started from
those values, bit for bit (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import spotgen
from parity import compare, summary

pytestmark = pytest.mark.gpu


def _up(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda:0"))


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    return np.array_equal(a, b, equal_nan=a.dtype.kind == "f")


def _agree(mine, ref64):
    """float32 results of a double-precision estimate summed in another order:
    equal, or one float32 rounding apart where the double sits on a boundary."""
    ref = ref64.astype(np.float32)
    same = (mine == ref) | (np.isnan(mine) & np.isnan(ref))
    rel = np.abs(mine.astype(np.float64) - ref64) / np.maximum(np.abs(ref64), 1e-30)
    return same.mean(), np.nanmax(np.where(same, 0.0, rel), initial=0.0)


def _usable(b, opts):
    w, h, m = (b.sizes[:, i].astype(int) for i in range(3))
    return ((w >= 3) & (h >= 3) & (np.maximum(w, h) <= opts.max_side) & (w * h <= opts.max_pixels)
            & ((m == spotgen.SYM) | (m == spotgen.ELL)))


def _check_init(raw, b, opts, min_frac=0.999):
    ok = _usable(b, opts)
    assert np.all(np.isnan(raw["init"][~ok]))
    if not ok.any():
        return ok
    frac, worst = _agree(raw["init"][ok], oracle.moment_init_batch(b.subset(np.flatnonzero(ok))))
    print(f"{frac:.6f} identical to the oracle, worst other rel diff {worst:.2e}")
    assert frac >= min_frac and worst <= 2.0 ** -23
    return ok


def _run(ctx, b, opts):
    import torch
    d = (_up(b.data), _up(b.sizes), _up(b.offsets))
    raw = ctx.fit_raw(*d, opts, want_evals=True)
    torch.cuda.synchronize()
    two = ctx.fit_spots(*d, raw["init"].clone(), opts, want_evals=True)
    alone = ctx.moment_init(*d, opts)
    torch.cuda.synchronize()
    return _host(raw), _host(two), alone.cpu().numpy()


CASES = [
    # workload, spots, options, start values bit for bit with spotfit_moment_init
    ("scale_15x15", 20000, dict(max_side=16), True),
    ("small_11x11", 3000, dict(max_side=16), True),
    ("precision_32x32_ell", 3000, dict(max_side=32), True),
    ("serve_fiducials", 4000, dict(max_side=32), True),
    ("mixed_7to32", 20000, dict(schedule=1), False),
    ("mixed_7to32", 20000, dict(schedule=1, plan_hint=1), False),
    ("scale_15x15", 5000, dict(max_side=16, plan_hint=1), False),
    ("small_11x11", 3000, dict(max_side=8, plan_hint=1), False),
    ("precision_32x32_ell", 2000, dict(max_side=32, plan_hint=1), False),
    ("mixed_7to32", 6000, dict(precision=0), True),
    ("scale_15x15", 3000, dict(max_side=16, precision=1), True),
    ("small_11x11", 1000, dict(max_side=16, precision=3), True),
]


@pytest.mark.parametrize("name,n,kw,bitwise_init", CASES,
                         ids=[f"{c[0]}-{'-'.join(f'{k}{v}' for k, v in c[2].items())}" for c in CASES])
def test_fit_raw_is_the_two_call_composition(name, n, kw, bitwise_init):
    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload(name, n=n)
    opts = sf.default_options(**kw)
    raw, two, alone = _run(ctx, b, opts)
    # the start values: the oracle's estimate, and the start-value kernel's
    _check_init(raw, b, opts)
    if bitwise_init:
        assert _same(raw["init"], alone)
    # the fit: what spotfit_fit_spots gives from the same start values
    for k in ("params", "chi2", "iters", "status", "evals"):
        assert _same(raw[k], two[k]), k


def test_fit_raw_decisions_match_the_oracle():
    """The oracle fit started from the start values the launch computed takes the
    same decisions."""
    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload("mixed_7to32", n=8000)
    opts = sf.default_options(schedule=sf.SCHEDULE_MIXED)
    raw, _, _ = _run(ctx, b, opts)
    b2 = spotgen.SpotBatch(b.data, b.sizes, b.offsets, raw["init"], b.truth, "fused init")
    r = oracle.fit_batch(b2, oracle.default_opts(), threads=8)
    c = compare(raw, r, chi_band=1e-11, step_band=1e-9)
    print(summary("fit_raw", c))
    assert c["strict_mismatch"] == 0 and c["tol_fail_same"] == 0


@pytest.mark.parametrize("n", [1, 5, 17, 33])
def test_fit_raw_small_batches_and_unusable_shapes(n):
    """Batches smaller than a chunk, ragged chunks, float data, and the shapes a
    fit rejects (NaN start values, BAD_INPUT)."""
    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload("mixed_7to32", n=n, seed=11 + n)
    f = spotgen.SpotBatch(b.data.astype(np.float32) * 0.5 + 3.0, b.sizes.copy(), b.offsets,
                          b.init, b.truth, "f32")
    f.sizes[0, 2] = 7                      # unknown model
    if n > 1:
        f.sizes[1, 0] = 2                  # too narrow
    for kw in (dict(max_side=16), dict(max_side=16, plan_hint=1), dict(schedule=1)):
        opts = sf.default_options(**kw)
        raw, two, alone = _run(ctx, f, opts)
        ok = _check_init(raw, f, opts, min_frac=0.99)
        assert not ok[0] and (n == 1 or not ok[1])
        assert np.all(raw["status"][~ok] == sf.BAD_INPUT)
        assert np.all(raw["status"][ok] != sf.BAD_INPUT)
        for k in ("params", "chi2", "iters", "status", "evals"):
            assert _same(raw[k], two[k]), (kw, k)


def test_fit_raw_zero_spots():
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    dev = torch.device("cuda:0")
    out = ctx.fit_raw(torch.zeros(0, dtype=torch.uint16, device=dev),
                      torch.zeros((0, 4), dtype=torch.uint8, device=dev),
                      torch.zeros(0, dtype=torch.int64, device=dev))
    assert out["init"].shape == (0, 4) and out["params"].shape == (0, 6)


def test_fit_raw_full_size_scale_workload():
    """1M spots of 15x15 in the benchmark's launch configuration: fit_raw gives
    spotfit_moment_init's start values and fit_spots' results bit for bit on
    every spot; a sample against the oracle's start values and fits."""
    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.config(1, threads=16)
    opts = sf.default_options(max_side=16)
    raw, two, alone = _run(ctx, b, opts)
    assert _same(raw["init"], alone)
    for k in ("params", "chi2", "iters", "status", "evals"):
        assert _same(raw[k], two[k]), k
    assert np.all(raw["status"] != sf.BAD_INPUT)
    idx = np.sort(np.random.default_rng(21).choice(b.n, size=3000, replace=False))
    sub = b.subset(idx)
    _check_init({"init": raw["init"][idx]}, sub, opts)
    s2 = spotgen.SpotBatch(sub.data, sub.sizes, sub.offsets, raw["init"][idx], sub.truth, "fused")
    r = oracle.fit_batch(s2, oracle.default_opts(), threads=8)
    c = compare({k: v[idx] for k, v in raw.items()}, r, chi_band=1e-11, step_band=1e-9)
    print(summary("fit_raw 1M sample", c))
    assert c["strict_mismatch"] == 0 and c["tol_fail_same"] == 0
