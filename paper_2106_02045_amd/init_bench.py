"""Start values on the device: time of the two start-value kernels against the
HBM roofline (each reads every pixel once).

    python -m paper_2106_02045_amd.init_bench [--workloads scale_15x15,precision_32x32_ell]

Per workload and method (moment: centroid / second moments; peak: the paper's
3x3 moving average, brightest pixel, sigma = sqrt(M/pi)): the kernel's average
time over 20 calls (HIP events on the stream), spots/s, and the algorithmic
bytes per call (pixels + 4 B shape + 8 B offset read, 16 B start values
written per spot) over that time against 8 TB/s.  One JSON line each.

With --raw: raw spots to fits, per workload: the fit alone from given start
values, the start-value kernel followed by the fit (two launches), and
spotfit_fit_raw (start values computed inside the fit's launch); average time
per call over --reps calls (HIP events on the stream).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="scale_15x15,precision_32x32_ell")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--raw", action="store_true", help="time raw spots to fits instead")
    ap.add_argument("--plan", choices=["throughput", "latency"], default="throughput")
    ap.add_argument("--spots", default="", help="with --raw: comma list of batch sizes "
                    "(the first spots of each workload; default: the whole workload)")
    a = ap.parse_args(argv)

    import torch

    import paper_2106_02045_amd as sf
    import spotgen

    dev = torch.device("cuda:0")
    ctx = sf.Context(0)
    st = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(a.reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / a.reps

    if a.raw:
        sizes = [int(x) for x in a.spots.split(",") if x] or [None]
        for name, n_spots in ((w, k) for w in a.workloads.split(",") for k in sizes):
            b = spotgen.workload(name, n=n_spots, threads=16)
            up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
            d = (up(b.data), up(b.sizes), up(b.offsets))
            side = int(max(b.sizes[:, 0].max(), b.sizes[:, 1].max()))
            uneven = len(np.unique(np.maximum(b.sizes[:, 0], b.sizes[:, 1]))) > 1
            opts = sf.default_options(
                max_side=max(3, side),
                schedule=sf.SCHEDULE_MIXED if uneven else sf.SCHEDULE_UNIFORM,
                plan_hint=sf.PLAN_LATENCY if a.plan == "latency" else sf.PLAN_THROUGHPUT)
            init = ctx.moment_init(*d, opts)
            out = ctx.fit_spots(*d, init, opts)
            out_raw = dict(out, init=torch.empty_like(init))
            t_fit = timed(lambda: ctx.fit_spots(*d, init, opts, out=out))
            t_two = timed(lambda: (ctx.moment_init(*d, opts, out=init),
                                   ctx.fit_spots(*d, init, opts, out=out)))
            t_raw = timed(lambda: ctx.fit_raw(*d, opts, out=out_raw))
            same = bool(torch.equal(out_raw["status"], out["status"]))
            print(json.dumps({"workload": name, "spots": b.n, "plan": a.plan,
                              "schedule": "mixed" if uneven else "uniform",
                              "fit_ms": t_fit, "init_then_fit_ms": t_two, "fit_raw_ms": t_raw,
                              "fits_per_s_raw": b.n / t_raw * 1e3,
                              "status_same_as_two_calls": same}), flush=True)
        return

    for name in a.workloads.split(","):
        b = spotgen.workload(name, threads=16)
        up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        d = (up(b.data), up(b.sizes), up(b.offsets))
        side = int(max(b.sizes[:, 0].max(), b.sizes[:, 1].max()))
        opts = sf.default_options(max_side=max(3, side))
        out = torch.empty((b.n, 4), dtype=torch.float32, device=dev)
        alg_bytes = float(b.data.nbytes + b.n * (4 + 8 + 16))
        for method, fn in (("moment", ctx.moment_init), ("peak", ctx.peak_init)):
            fn(*d, opts, out=out)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(a.reps):
                fn(*d, opts, out=out)
            e1.record(st)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / a.reps
            gbps = alg_bytes / t / 1e9
            print(json.dumps({"workload": name, "method": method, "spots": b.n,
                              "kernel_ms": t * 1e3, "spots_per_s": b.n / t,
                              "alg_bytes_per_call": alg_bytes, "achieved_GBps": gbps,
                              "frac_hbm": gbps / PEAK_HBM_GBPS,
                              "bad": int(np.isnan(out[:, 0].cpu().numpy()).sum())}), flush=True)


if __name__ == "__main__":
    main()
