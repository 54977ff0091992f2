"""Captured fits of fixed-shape batches (spotfit_graph_*), through the C ABI
(needs an MI355X): every replay gives the bits of a direct call on the same
inputs, with the program's own eager work and synchronisations between replays."""
import numpy as np
import pytest

import spotgen

pytestmark = pytest.mark.gpu


def _up(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda:0"))


def _direct(ctx, b, opts):
    import torch
    out = ctx.fit_spots(_up(b.data), _up(b.sizes), _up(b.offsets), _up(b.init), opts)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _eager_noise():
    import torch
    x = torch.arange(100000, device="cuda:0", dtype=torch.float32)
    return float((x * 0.5).sum().item())


@pytest.mark.parametrize("plan", ["throughput", "latency"])
def test_graph_replays_equal_direct_fits(plan):
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    _, _, frames = spotgen.drift_frames(6, n_markers=32, side=13, seed=31)
    opts = sf.default_options(max_side=13, plan_hint=sf.PLAN_LATENCY if plan == "latency"
                              else sf.PLAN_THROUGHPUT)
    f0 = frames[0]
    d = dict(data=_up(f0.data), sizes=_up(f0.sizes), offsets=_up(f0.offsets), init=_up(f0.init))
    g = ctx.graph(d["data"], d["sizes"], d["offsets"], d["init"], opts)
    for f in frames:
        d["data"].copy_(torch.from_numpy(f.data))
        d["init"].copy_(torch.from_numpy(f.init))
        for t in g.out.values():
            t.fill_(-1)
        _eager_noise()
        g.launch()
        torch.cuda.synchronize()
        want = _direct(ctx, f, opts)
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(g.out[k].cpu().numpy(), want[k])
    g.close()


def test_graph_with_host_copies():
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    _, _, frames = spotgen.drift_frames(5, n_markers=24, side=11, seed=32)
    opts = sf.default_options(max_side=11)
    f0 = frames[0]
    n = f0.n
    d = dict(data=_up(f0.data), sizes=_up(f0.sizes), offsets=_up(f0.offsets), init=_up(f0.init))
    host = dict(data=torch.empty(f0.data.shape, dtype=torch.uint16).pin_memory(),
                init=torch.empty((n, 4), dtype=torch.float32).pin_memory(),
                params=torch.empty((n, 6), dtype=torch.float32).pin_memory(),
                chi2=torch.empty(n, dtype=torch.float32).pin_memory(),
                iters=torch.empty(n, dtype=torch.int32).pin_memory(),
                status=torch.empty(n, dtype=torch.int32).pin_memory())
    g = ctx.graph(d["data"], d["sizes"], d["offsets"], d["init"], opts, host=host)
    for f in frames:
        host["data"].copy_(torch.from_numpy(f.data))
        host["init"].copy_(torch.from_numpy(f.init))
        for k in ("params", "chi2", "iters", "status"):
            host[k].fill_(-1)
        _eager_noise()
        g.launch()
        torch.cuda.synchronize()
        want = _direct(ctx, f, opts)
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(host[k].numpy(), want[k])
    g.close()


def test_graph_mixed_schedule():
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload("mixed_7to32", n=3000)
    opts = sf.default_options(schedule=sf.SCHEDULE_MIXED)
    d = dict(data=_up(b.data), sizes=_up(b.sizes), offsets=_up(b.offsets), init=_up(b.init))
    g = ctx.graph(d["data"], d["sizes"], d["offsets"], d["init"], opts)
    want = _direct(ctx, b, opts)
    for _ in range(3):
        for t in g.out.values():
            t.zero_()
        _eager_noise()
        g.launch()
        torch.cuda.synchronize()
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(g.out[k].cpu().numpy(), want[k])
    g.close()


def test_graph_mixed_schedule_survives_workspace_growth():
    """The graph keeps its own mixed-schedule workspace: growing the context's
    (a larger mixed call, an explicit reserve) between replays changes nothing."""
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload("mixed_7to32", n=2000)
    big = spotgen.workload("mixed_7to32", n=30000, seed=77)
    opts = sf.default_options(schedule=sf.SCHEDULE_MIXED)
    d = dict(data=_up(b.data), sizes=_up(b.sizes), offsets=_up(b.offsets), init=_up(b.init))
    g = ctx.graph(d["data"], d["sizes"], d["offsets"], d["init"], opts)
    want = _direct(ctx, b, opts)
    for step in range(3):
        if step == 1:
            _direct(ctx, big, opts)      # grows the context's workspace
        if step == 2:
            ctx.reserve(200000)          # and again
        for t in g.out.values():
            t.zero_()
        _eager_noise()
        g.launch()
        torch.cuda.synchronize()
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(g.out[k].cpu().numpy(), want[k])
    g.close()


@pytest.mark.parametrize("kw", [dict(max_side=13), dict(max_side=13, plan_hint=1),
                                dict(schedule=1), dict(max_side=13, precision=0)],
                         ids=["throughput", "latency", "mixed", "fp32"])
def test_graph_of_raw_frames(kw):
    """init None: every replay takes the pinned pixels of a frame to fits, start
    values computed on the device; the bits of a direct fit_raw call."""
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    _, _, frames = spotgen.drift_frames(5, n_markers=40, side=13, seed=33)
    opts = sf.default_options(**kw)
    f0 = frames[0]
    n = f0.n
    d = dict(data=_up(f0.data), sizes=_up(f0.sizes), offsets=_up(f0.offsets))
    host = dict(data=torch.empty(f0.data.shape, dtype=torch.uint16).pin_memory(),
                params=torch.empty((n, 6), dtype=torch.float32).pin_memory(),
                chi2=torch.empty(n, dtype=torch.float32).pin_memory(),
                iters=torch.empty(n, dtype=torch.int32).pin_memory(),
                status=torch.empty(n, dtype=torch.int32).pin_memory())
    g = ctx.graph(d["data"], d["sizes"], d["offsets"], None, opts, host=host)
    for f in frames:
        host["data"].copy_(torch.from_numpy(f.data))
        for k in ("params", "chi2", "iters", "status"):
            host[k].fill_(-1)
        _eager_noise()
        g.launch()
        torch.cuda.synchronize()
        want = ctx.fit_raw(_up(f.data), _up(f.sizes), _up(f.offsets), opts)
        torch.cuda.synchronize()
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(host[k].numpy(), want[k].cpu().numpy())
        assert np.all(host["status"].numpy() != sf.BAD_INPUT)
    g.close()
