"""spotfit_fit_spots_noalloc through the C ABI (needs an MI355X): its fits equal
those of spotfit_fit_spots bit for bit, on two calls in a row whose second is
smaller (so stale counters or lists of the shared scratch array would show), for
the uniform and the mixed schedule and both plan hints; mixed-schedule calls
beyond the array's capacity are refused before any work is queued."""
import numpy as np
import pytest

import spotgen

pytestmark = pytest.mark.gpu

KEYS = ("params", "chi2", "iters", "status", "evals")


def _up(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda:0"))


def _outs(n):
    import torch
    dev = torch.device("cuda:0")
    return dict(params=torch.full((n, 6), float("nan"), device=dev),
                chi2=torch.full((n,), -1.0, device=dev),
                iters=torch.full((n,), -7, dtype=torch.int32, device=dev),
                status=torch.full((n,), -7, dtype=torch.int32, device=dev),
                evals=torch.full((n, 2), -7, dtype=torch.int32, device=dev))


def _fit(ctx, b, opts, noalloc):
    import torch
    d = (_up(b.data), _up(b.sizes), _up(b.offsets), _up(b.init))
    out = _outs(b.n)
    f = ctx.fit_spots_noalloc if noalloc else ctx.fit_spots
    f(*d, opts, out=out)
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy() for k in KEYS}


CASES = [
    ("scale_15x15", "uniform", "throughput", 40000, 7000),
    ("scale_15x15", "uniform", "latency", 3000, 500),
    ("mixed_7to32", "mixed", "throughput", 90000, 20000),  # > 65536: separate reset + classify
    ("mixed_7to32", "mixed", "latency", 30000, 4000),
    ("precision_32x32_ell", "uniform", "throughput", 6000, 1500),
]


@pytest.mark.parametrize("name,schedule,hint,n1,n2", CASES)
def test_noalloc_equals_fit_spots(name, schedule, hint, n1, n2):
    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    big = spotgen.workload(name, n=n1)
    rng = np.random.default_rng(5)
    small = big.subset(np.sort(rng.choice(n1, size=n2, replace=False)))
    max_side = int(big.sizes[:, :2].max())
    opts = sf.default_options(max_side=max_side, max_pixels=max(9, int(big.npix().max())),
                              schedule=sf.SCHEDULE_MIXED if schedule == "mixed" else
                              sf.SCHEDULE_UNIFORM,
                              plan_hint=sf.PLAN_LATENCY if hint == "latency" else
                              sf.PLAN_THROUGHPUT)
    for b in (big, small):  # two calls in a row, the second on fewer spots
        print(f"case {name} {schedule} {hint} n={b.n}", flush=True)
        got = _fit(ctx, b, opts, True)
        want = _fit(ctx, b, opts, False)
        assert (got["status"] >= 0).all() and (got["iters"] >= 0).all()
        for k in KEYS:
            np.testing.assert_array_equal(got[k], want[k], err_msg=k)


def test_noalloc_mixed_capacity_refused():
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    n = sf.NOALLOC_MAX_SPOTS + 1
    dev = torch.device("cuda:0")
    data = torch.zeros(9 * n, dtype=torch.uint16, device=dev)
    sizes = torch.tensor([3, 3, 0, 0], dtype=torch.uint8, device=dev).repeat(n, 1)
    offs = torch.arange(n, dtype=torch.int64, device=dev) * 9
    init = torch.tensor([1.0, 1.0, 1.0, 1.0], device=dev).repeat(n, 1)
    out = _outs(n)
    opts = sf.default_options(max_side=3, schedule=sf.SCHEDULE_MIXED)
    with pytest.raises(sf.SpotfitError):
        ctx.fit_spots_noalloc(data, sizes, offs, init, opts, out=out)
    torch.cuda.synchronize()
    assert int(out["iters"].min().item()) == -7  # nothing was written
    # the uniform schedule takes the same batch
    opts_u = sf.default_options(max_side=3)
    ctx.fit_spots_noalloc(data, sizes, offs, init, opts_u, out=out)
    torch.cuda.synchronize()
    assert int(out["status"].max().item()) <= sf.BAD_INPUT and int(out["status"].min().item()) >= 0
