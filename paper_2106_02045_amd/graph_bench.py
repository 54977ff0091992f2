"""Per-frame call time for fixed-shape frames: a direct call sequence against
one replay of a captured graph.

    python -m paper_2106_02045_amd.graph_bench [--frames 5000] [--markers 32]

Each frame holds the same markers (13x13 ROIs) of a drifting sample.  Direct:
copy the frame's pixels and start values from pinned host memory, fit, copy the
results back, synchronise.  Graph: the same sequence captured once
(spotfit_graph_create with host copies) and replayed with one launch per frame.
Prints one JSON line per (plan, mode) with p50 / p99 of the per-frame time.
With --raw the frames carry no start values: direct calls spotfit_fit_raw and
the graph is captured with init NULL (start values computed on the device).
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=5000)
    ap.add_argument("--markers", type=int, default=32)
    ap.add_argument("--raw", action="store_true", help="frames without start values")
    a = ap.parse_args(argv)

    import torch

    import paper_2106_02045_amd as sf
    import spotgen

    dev = torch.device("cuda:0")
    ctx = sf.Context(0)
    _, _, frames = spotgen.drift_frames(64, n_markers=a.markers, side=13, seed=5)
    f0 = frames[0]
    n = f0.n
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    d = dict(data=up(f0.data), sizes=up(f0.sizes), offsets=up(f0.offsets), init=up(f0.init))
    host = dict(data=torch.empty(f0.data.shape, dtype=torch.uint16).pin_memory(),
                init=torch.empty((n, 4), dtype=torch.float32).pin_memory(),
                params=torch.empty((n, 6), dtype=torch.float32).pin_memory(),
                chi2=torch.empty(n, dtype=torch.float32).pin_memory(),
                iters=torch.empty(n, dtype=torch.int32).pin_memory(),
                status=torch.empty(n, dtype=torch.int32).pin_memory())
    if a.raw:
        del host["init"]
    st = torch.cuda.current_stream(dev)
    for plan in ("latency", "throughput"):
        opts = sf.default_options(max_side=13, plan_hint=sf.PLAN_LATENCY if plan == "latency"
                                  else sf.PLAN_THROUGHPUT)
        out = {k: torch.empty_like(v, device=dev) for k, v in host.items()
               if k in ("params", "chi2", "iters", "status")}
        g = ctx.graph(d["data"], d["sizes"], d["offsets"], None if a.raw else d["init"], opts,
                      out=out, host=host)

        def direct():
            d["data"].copy_(host["data"], non_blocking=True)
            if a.raw:
                ctx.fit_raw(d["data"], d["sizes"], d["offsets"], opts, out=dict(out, init=d["init"]))
            else:
                d["init"].copy_(host["init"], non_blocking=True)
                ctx.fit_spots(d["data"], d["sizes"], d["offsets"], d["init"], opts, out=out)
            for k in out:
                host[k].copy_(out[k], non_blocking=True)
            torch.cuda.synchronize()

        def graph():
            g.launch(st)
            torch.cuda.synchronize()

        for mode, call in (("direct", direct), ("graph", graph)):
            ts = []
            for i in range(a.frames):
                f = frames[i % len(frames)]
                host["data"].copy_(torch.from_numpy(f.data))
                if not a.raw:
                    host["init"].copy_(torch.from_numpy(f.init))
                t0 = time.perf_counter()
                call()
                ts.append(time.perf_counter() - t0)
            ts = np.asarray(ts[50:]) * 1e6
            print(json.dumps({"plan": plan, "mode": mode, "markers": n, "frames": len(ts),
                              "start_values": "device" if a.raw else "host",
                              "p50_us": float(np.percentile(ts, 50)),
                              "p99_us": float(np.percentile(ts, 99)),
                              "mean_us": float(ts.mean())}), flush=True)
        g.close()


if __name__ == "__main__":
    main()
