"""Accuracy of the fitted shaping parameters on the paper's simulated spots
(Results section, Table 1, and the supplementary figures): every fit on the
device, from the paper's own start values computed on the device.

    python -m paper_2106_02045_amd.accuracy_bench [--fits 100000]

Cases: the three Table 1 rows (9x9 pixels; 400:40, 1600:40 and 1600:0 signal to
background counts) and the supplementary grid (7x7, 9x9, 11x11 pixels; 160, 400
and 1000 signal counts; one background count per pixel).  Spots follow the
paper's protocol (centre normal around the ROI centre with sd S/20, sigma
U[1, 2], Gaussian noise of variance equal to the intensity, rounded to
non-negative integers).  Errors are absolute and in units of sigma_true:
median, mean and std of |x - x_true|, |y - y_true| (pooled) and of
|sigma - sigma_true|, beside sigma_true / sqrt(N_signal), the mean error
expected at best without background.  Prints one JSON line per case.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TABLE1 = [(9, 400, 40), (9, 1600, 40), (9, 1600, 0)]
SUPPLEMENT = [(S, sig, S * S) for S in (7, 9, 11) for sig in (160, 400, 1000)]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fits", type=int, default=100000)
    ap.add_argument("--seed", type=int, default=50)
    a = ap.parse_args(argv)

    import torch

    import paper_2106_02045_amd as sf
    import spotgen

    dev = torch.device("cuda:0")
    ctx = sf.Context(0)
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    for group, cases in (("table1", TABLE1), ("supplement", SUPPLEMENT)):
        for S, n_sig, n_bg in cases:
            b = spotgen.paper_protocol(a.fits, S, float(n_sig), float(n_bg), seed=a.seed)
            d = (up(b.data), up(b.sizes), up(b.offsets))
            o = sf.default_options(max_side=max(S, 3))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            init = ctx.peak_init(*d, o)
            out = ctx.fit_spots(*d, init, o)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            p = out["params"].cpu().numpy().astype(np.float64)
            status = out["status"].cpu().numpy()
            iters = out["iters"].cpu().numpy()
            t = b.truth
            exy = np.concatenate([np.abs(p[:, 0] - t[:, 0]), np.abs(p[:, 1] - t[:, 1])]) / \
                np.tile(t[:, 2], 2)
            es = np.abs(p[:, 2] - t[:, 2]) / t[:, 2]
            print(json.dumps({
                "group": group, "S": S, "n_signal": n_sig, "n_background": n_bg, "fits": b.n,
                "xy": [float(np.median(exy)), float(exy.mean()), float(exy.std())],
                "sigma": [float(np.median(es)), float(es.mean()), float(es.std())],
                "bound_mean": 1.0 / math.sqrt(n_sig),
                "status_frac": (np.bincount(status, minlength=6) / b.n).tolist(),
                "iters_mean": float(iters.mean()),
                "device_s": dt,
            }), flush=True)


if __name__ == "__main__":
    main()
