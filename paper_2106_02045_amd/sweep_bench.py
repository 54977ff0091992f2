"""Execution time against image size and batch size (the paper's Results section,
Figs. 2-4): S x S spots for S = 4..32, batches of 10 to 10'000 fits per call.

    python -m paper_2106_02045_amd.sweep_bench [--sizes 4-32] [--batches 10,100,1000,10000]

Spots follow the paper's timing protocol: centre normal around the ROI centre with
sd S/20, sigma U[1, 2], integrated signal 400, total background 40 spread over the
ROI, Gaussian noise of variance equal to the intensity, rounded to non-negative
integers; start values by the paper's recipe, computed once outside the timing.
As in the paper, one timed call transfers the batch from host memory (pinned
here), fits it and copies the results back; the kernel-only time (HIP events on
the stream) is reported beside it.  Batches of 10, 100, 1000 and 10000 fits run
200, 50, 20 and 10 times.  Prints one JSON line per (S, batch).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

REPS = {10: 200, 100: 50, 1000: 20, 10000: 10}


def _sizes(spec: str):
    out = []
    for part in spec.split(","):
        if "-" in part:
            a, b = part.split("-")
            out += list(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="4-32")
    ap.add_argument("--batches", default="10,100,1000,10000")
    ap.add_argument("--plan", default="throughput", choices=["throughput", "latency"],
                    help="lane mapping: few lanes per spot, or one lane per column")
    a = ap.parse_args(argv)

    import torch

    import paper_2106_02045_amd as sf
    import spotgen

    dev = torch.device("cuda:0")
    ctx = sf.Context(0)
    st = torch.cuda.current_stream(dev)
    batches = [int(b) for b in a.batches.split(",")]
    nmax = max(batches)
    for S in _sizes(a.sizes):
        full = spotgen.paper_protocol(nmax, S, 400.0, 40.0, seed=21, init="paper")
        opts = sf.default_options(max_side=max(S, 3),
                                  plan_hint=(sf.PLAN_LATENCY if a.plan == "latency"
                                             else sf.PLAN_THROUGHPUT))
        for B in batches:
            b = full.subset(np.arange(B))
            host = dict(data=torch.from_numpy(np.ascontiguousarray(b.data)).pin_memory(),
                        sizes=torch.from_numpy(np.ascontiguousarray(b.sizes)).pin_memory(),
                        offsets=torch.from_numpy(np.ascontiguousarray(b.offsets)).pin_memory(),
                        init=torch.from_numpy(np.ascontiguousarray(b.init)).pin_memory())
            dv = {k: torch.empty_like(v, device=dev) for k, v in host.items()}
            outs = dict(params=torch.empty((B, 6), dtype=torch.float32, device=dev),
                        chi2=torch.empty(B, dtype=torch.float32, device=dev),
                        iters=torch.empty(B, dtype=torch.int32, device=dev),
                        status=torch.empty(B, dtype=torch.int32, device=dev))
            res = {k: torch.empty(v.shape, dtype=v.dtype).pin_memory() for k, v in outs.items()}

            def call():
                for k in host:
                    dv[k].copy_(host[k], non_blocking=True)
                ctx.fit_spots(dv["data"], dv["sizes"], dv["offsets"], dv["init"], opts, out=outs)
                for k in outs:
                    res[k].copy_(outs[k], non_blocking=True)
                torch.cuda.synchronize()

            call()  # warm-up
            reps = REPS.get(B, 10)
            t0 = time.perf_counter()
            for _ in range(reps):
                call()
            e2e = (time.perf_counter() - t0) / reps
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                ctx.fit_spots(dv["data"], dv["sizes"], dv["offsets"], dv["init"], opts, out=outs)
            e1.record(st)
            torch.cuda.synchronize()
            kern = e0.elapsed_time(e1) / 1e3 / reps
            status = res["status"].numpy()
            print(json.dumps({
                "S": S, "batch": B, "reps": reps, "plan": a.plan,
                "end_to_end_s": e2e, "fits_per_s": B / e2e, "pixels_per_s": B * S * S / e2e,
                "kernel_s": kern, "kernel_fits_per_s": B / kern,
                "bad_input": int((status == 5).sum()),
            }), flush=True)


if __name__ == "__main__":
    main()
