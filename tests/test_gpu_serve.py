"""Mixed-size schedule and the serving loop, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import spotgen
from parity import compare, summary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import paper_2106_02045_amd as m
    return m


def _fit(sf, ctx, b, opts):
    import torch
    dev = torch.device("cuda:0")
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    out = ctx.fit_spots(up(b.data), up(b.sizes), up(b.offsets), up(b.init), opts, want_evals=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_mixed_schedule_matches_oracle_and_uniform(sf):
    ctx = sf.Context(0)
    b = spotgen.config(3, n=30000)
    gm = _fit(sf, ctx, b, sf.default_options(schedule=sf.SCHEDULE_MIXED))
    r = oracle.fit_batch(b, oracle.default_opts(), threads=8)
    c = compare(gm, r, chi_band=1e-11, step_band=1e-9)
    print(summary("mixed schedule 30k", c))
    assert c["strict_mismatch"] == 0 and c["tol_fail_same"] == 0
    # every spot's result is independent of how the batch was scheduled
    for side in (8, 16, 32):
        sel = np.nonzero(np.maximum(b.sizes[:, 0], b.sizes[:, 1]) <= side)[0]
        sel = sel[np.maximum(b.sizes[sel, 0], b.sizes[sel, 1]) > side // 2]
        sub = b.subset(sel)
        gu = _fit(sf, ctx, sub, sf.default_options(max_side=side))
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(gu[k], gm[k][sel])


def test_mixed_schedule_workspace_reuse_and_growth(sf):
    ctx = sf.Context(0)
    ctx.reserve(100)
    o = sf.default_options(schedule=sf.SCHEDULE_MIXED)
    b1 = spotgen.config(3, n=5000)
    b2 = spotgen.config(3, n=700, seed=9)
    g1 = _fit(sf, ctx, b1, o)        # grows the workspace
    g2 = _fit(sf, ctx, b2, o)        # smaller call reuses it
    g1b = _fit(sf, ctx, b1, o)
    for k in g1:
        np.testing.assert_array_equal(g1[k], g1b[k])
    assert np.all(g2["status"] != 5)


def test_serving_alone_equals_mix_and_oracle(sf):
    ts, frames = spotgen.serve_frames(300, fps=5000.0, seed=7, threads=8)
    opts = sf.default_options(max_side=21, schedule=sf.SCHEDULE_MIXED)
    srv = sf.Server(0, opts, device_mem_budget=64 << 20, max_frames=512, n_streams=3)
    offs = np.round((ts - ts[0]) * 1e9).astype(np.uint64)
    outs = srv.replay([(f.data, f.sizes, f.init) for f in frames], offs)
    st = srv.stats()
    srv.close()
    print("serve stats", st)
    assert st["frames_done"] == len(frames) and st["frames_failed"] == 0
    assert st["spots_done"] == sum(f.n for f in frames)
    ctx = sf.Context(0)
    for f in range(0, len(frames), 37):
        alone = _fit(sf, ctx, frames[f], opts)
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(alone[k], outs[f][k])
    # and against the oracle
    allb = frames[0]
    r = oracle.fit_batch(allb, oracle.default_opts(), threads=4)
    c = compare(outs[0], r, chi_band=1e-11, step_band=1e-9)
    assert c["strict_mismatch"] == 0 and c["tol_fail_same"] == 0


def test_serving_admission_by_memory(sf):
    # a budget that holds only a few frames: submit refuses, then admits once
    # earlier frames complete; every frame still finishes correctly
    ts, frames = spotgen.serve_frames(60, fps=1e6, seed=8, threads=4)
    opts = sf.default_options(max_side=21)
    srv = sf.Server(0, opts, device_mem_budget=1 << 20, max_frames=4, n_streams=2)
    import time
    pending = []
    refused = 0
    for f in frames:
        while True:
            r = srv.submit(f.data, f.sizes, f.init)
            if r is not None:
                pending.append(r)
                break
            refused += 1
            time.sleep(2e-4)
    results = [srv.wait(t) for t, _ in pending]
    st = srv.stats()
    srv.close()
    assert st["frames_done"] == len(frames)
    assert refused > 0 and st["rejected"] == refused
    ctx = sf.Context(0)
    alone = _fit(sf, ctx, frames[11], opts)
    np.testing.assert_array_equal(alone["params"], results[11]["params"])


def test_serving_reports_a_failed_frame_after_its_release(sf, monkeypatch):
    """A frame whose batch fails stays failed: wait() raises for it, also once its
    ring space has been released and reused, and the other frames complete.  The
    failure is forced on the host (the second batch is not enqueued at all)."""
    monkeypatch.setenv("SPOTFIT_SERVE_FAIL_BATCH", "2")
    ts, frames = spotgen.serve_frames(40, fps=1000.0, seed=12, threads=4)
    opts = sf.default_options(max_side=21)
    srv = sf.Server(0, opts, device_mem_budget=1 << 20, max_frames=4, n_streams=1)
    tickets = []
    for i, f in enumerate(frames[:3]):
        r = srv.submit(f.data, f.sizes, f.init)
        assert r is not None
        tickets.append(r[0])
        if i == 1:
            with pytest.raises(sf.SpotfitError, match="injected failure"):
                srv.wait(r[0])
        else:
            srv.wait(r[0])
    # more frames than slots: the failed frame's slot and ring space are reused
    import time
    for f in frames[3:]:
        while srv.submit(f.data, f.sizes, f.init) is None:
            time.sleep(2e-4)
    for t in range(tickets[-1] + 1, tickets[-1] + 1 + len(frames) - 3):
        srv.wait(t)
    assert srv.poll(tickets[1]) < 0
    assert srv.poll(tickets[0]) == 0 and srv.poll(tickets[2]) == 0
    st = srv.stats()
    srv.close()
    assert st["frames_failed"] == 1 and st["frames_done"] == len(frames) - 1


def test_serving_with_device_start_values(sf):
    # frames without start values: the loop computes them on the device, inside
    # the fit's launch; the results equal a direct fit_raw of the same spots, bit
    # for bit, and the fit from those start values
    import torch
    ts, frames = spotgen.serve_frames(120, fps=5000.0, seed=11, threads=8)
    opts = sf.default_options(max_side=21, schedule=sf.SCHEDULE_MIXED)
    srv = sf.Server(0, opts, device_mem_budget=64 << 20, max_frames=256, n_streams=2)
    offs = np.round((ts - ts[0]) * 1e9).astype(np.uint64)
    outs = srv.replay([(f.data, f.sizes, None) for f in frames], offs)
    st = srv.stats()
    srv.close()
    assert st["frames_done"] == len(frames) and st["frames_failed"] == 0
    ctx = sf.Context(0)
    dev = torch.device("cuda:0")
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    for f in range(0, len(frames), 17):
        b = frames[f]
        d = (up(b.data), up(b.sizes), up(b.offsets))
        g = ctx.fit_raw(*d, opts)
        g2 = ctx.fit_spots(*d, g["init"], opts)
        torch.cuda.synchronize()
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(g[k].cpu().numpy(), outs[f][k])
            np.testing.assert_array_equal(g2[k].cpu().numpy(), outs[f][k])


def test_latency_plan_in_serving_matches_direct_calls(sf):
    # the latency hint (one lane per column) in the serving loop and in direct calls:
    # identical bits, and the oracle's decisions
    ts, frames = spotgen.serve_frames(80, fps=5000.0, seed=12, threads=8)
    opts = sf.default_options(max_side=21, schedule=sf.SCHEDULE_MIXED, plan_hint=sf.PLAN_LATENCY)
    srv = sf.Server(0, opts, device_mem_budget=64 << 20, max_frames=256, n_streams=2)
    offs = np.round((ts - ts[0]) * 1e9).astype(np.uint64)
    outs = srv.replay([(f.data, f.sizes, f.init) for f in frames], offs)
    srv.close()
    ctx = sf.Context(0)
    for f in range(0, len(frames), 13):
        alone = _fit(sf, ctx, frames[f], opts)
        for k in ("params", "chi2", "iters", "status"):
            np.testing.assert_array_equal(alone[k], outs[f][k])
    r = oracle.fit_batch(frames[0], oracle.default_opts(), threads=4)
    c = compare(outs[0], r, chi_band=1e-11, step_band=1e-9)
    assert c["strict_mismatch"] == 0 and c["tol_fail_same"] == 0


def _drift_close(gpu, ref):
    """float32 roundings of two double-precision means summed in different orders:
    equal or one float32 step apart (NaN where the oracle has NaN)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(gpu), nan)
    step = np.spacing(np.abs(ref[~nan]).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(gpu[~nan] - ref[~nan]) <= 1.01 * step + 1e-12)


@pytest.mark.parametrize("fps,streams", [(1000.0, 1), (40000.0, 3)])
def test_drift_tracking_matches_oracle(sf, fps, streams):
    # markers of a drifting sample fitted in the serving loop; the device's drift
    # records against the oracle's drift over the same fitted positions, and the
    # tracked drift against the true one
    ref, drift, frames = spotgen.drift_frames(400, n_markers=32, side=13, seed=21)
    ref = ref.astype(np.float32)  # the reference as the library holds it
    # a few frames with markers that cannot be used: an unknown model (BAD_INPUT)
    for f in (5, 6, 250):
        frames[f].sizes[3:9, 2] = 7
    frames[7].sizes[:, 2] = 7  # no usable marker at all
    opts = sf.default_options(max_side=13, schedule=sf.SCHEDULE_MIXED, plan_hint=sf.PLAN_LATENCY)
    srv = sf.Server(0, opts, device_mem_budget=64 << 20, max_frames=512, n_streams=streams)
    window = 16
    srv.track(ref, window)
    offs = np.round(np.arange(len(frames)) / fps * 1e9).astype(np.uint64)
    outs = srv.replay([(f.data, f.sizes, f.init, True) for f in frames], offs)
    st = srv.stats()
    # a tracked frame must hold one spot per marker
    with pytest.raises(sf.SpotfitError):
        srv.submit(frames[0].data[:13 * 13 * 31], frames[0].sizes[:31], frames[0].init[:31],
                   track=True)
    srv.close()
    print("serve stats", st)
    assert st["frames_done"] == len(frames) and st["frames_failed"] == 0
    P = np.stack([o["params"] for o in outs])
    S = np.stack([o["status"] for o in outs])
    exp = oracle.drift_track(P, S, ref, window)
    got = np.concatenate([o["drift"] for o in outs])
    _drift_close(got["dx"], exp[:, 0])
    _drift_close(got["dy"], exp[:, 1])
    _drift_close(got["mean_dx"], exp[:, 2])
    _drift_close(got["mean_dy"], exp[:, 3])
    np.testing.assert_array_equal(got["n_used"], exp[:, 4].astype(np.int32))
    np.testing.assert_array_equal(got["n_frames"], exp[:, 5].astype(np.int32))
    assert got["n_used"][7] == 0 and 20 <= got["n_used"][5] <= 26 and got["n_frames"][7] > 0
    # the tracked drift follows the true drift (window mean of the truth)
    tw = np.stack([drift[max(0, f - window + 1):f + 1].mean(axis=0) for f in range(len(frames))])
    err = np.stack([got["mean_dx"], got["mean_dy"]], axis=1) - tw
    rms = np.sqrt(np.mean(err[window:] ** 2))
    print(f"tracked drift rms error {rms:.4f} px")
    assert rms < 0.01
