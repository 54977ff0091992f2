#!/usr/bin/env python3
"""Throughput benchmark of the batched Gaussian-spot fit on one MI355X.

One step = one call of spotfit_fit_spots over the whole workload (every spot
fitted to completion), inputs resident in HBM.  Default workload: 1,000,000
spots of 15x15 uint16 pixels, symmetric Gaussian, sigma U[1,3], amplitude
log-uniform [1e2, 1e4], background U[10, 200], Poisson plus read noise (sd 2).

Prints one JSON line: fits/s (whole job), the fit kernel's roofline figures
measured live with HIP events on the launch stream, and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak of this chip for single-lane FP32 / FP64 FMA: 256 CUs x 4 SIMD x 16 lanes
# x 2 flop x 2.4 GHz.  (The 157.3 TFLOP/s FP32 figure needs packed FP32
# instructions, which the library's kernels are compiled without.)
PEAK_ALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBPS = 8000.0
CLOCK_HZ = 2.4e9  # peak engine clock

# Algorithmic work per spot of N pixels with n_g derivative and n_t trial
# evaluations: N * (C_g n_g + C_t n_t - 11 (n_g - 1)) flop, exp count N (n_t + 1).
C_GRAD = {0: 66, 1: 88}
C_TRIAL = 16


# the source of the fit kernel that the default workload runs (the lane-owned
# kernel for spots up to 16 x 16) and the headers its code comes from
FIT_KERNEL_SOURCES = ("spotfit_owned.hip", "spotfit_owned.h", "separable.h", "spotfit_internal.h",
                      "spotfit_lm.h", "lanegroup.h", "xlane.h")


def kernel_source_hash() -> str:
    """sha256 over the sources the fit kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_02045_amd", "csrc")
    for name in FIT_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, schedule: str):
    """HBM bytes per launch of the fit kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a copy of known size), or None when
    no summary exists for this configuration or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}_{schedule}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t["hbm_bytes_per_launch"]


def measured_counters(workload: str, precision: str, schedule: str):
    """Per-launch hardware counters of the fit kernel from the committed summary
    (rocprofv3 --pmc over one launch), or None when no summary exists for this
    configuration or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}_{precision}_{schedule}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != kernel_source_hash():
        return None
    t["_path"] = path
    return t


def host_cpu() -> dict:
    """Logical CPUs of the host, those this process may run on, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return {"nproc": os.cpu_count(), "allowed": allowed, "model": model}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale_15x15")
    ap.add_argument("--n", type=int, default=None, help="spots (default: the workload's size)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "fp32", "plain", "comp"])
    ap.add_argument("--tie-tau", type=float, default=0.0)
    ap.add_argument("--schedule", default="uniform", choices=["uniform", "mixed", "per-size"],
                    help="uniform: one lane-group width for the batch; mixed: one persistent "
                         "launch with per-size-class widths; per-size: one launch per ROI side "
                         "(spots grouped by side on the host before timing)")
    ap.add_argument("--cpu-sample", type=int, default=1000000,
                    help="spots of the same workload fitted by the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the oracle's timed run (default: the host's cores, at most 16)")
    ap.add_argument("--pmc-copy-mb", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB once: the "
                         "calibration dispatch for hardware traffic counters")
    ap.add_argument("--parity-sample", type=int, default=2000,
                    help="spots compared with the CPU oracle after the timed run (0: none)")
    ap.add_argument("--serve-frames", type=int, default=10000,
                    help="after the timed fit steps, replay this many camera frames of the "
                         "serving workload at --serve-fps (Poisson arrivals) through the "
                         "serving loop and report their latency (0: skip)")
    ap.add_argument("--serve-fps", type=float, default=1000.0)
    ap.add_argument("--e2e-reps", type=int, default=5,
                    help="after the timed steps, this many end-to-end calls: pinned host inputs to "
                         "the device, the fit, results back to pinned host memory (0: skip)")
    ap.add_argument("--cpu-sample-1t", type=int, default=30000,
                    help="spots of the same workload fitted by the oracle on one thread")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {a.gpus}); the fit shards by "
              "independent spots, so N GPUs would each run this same benchmark on 1/N of "
              "the spots.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2106_02045_amd as sf
    import spotgen

    t0 = time.time()
    batch = spotgen.workload(a.workload, n=a.n, threads=16)
    gen_s = time.time() - t0
    n = batch.n
    npix = batch.npix()
    max_px = int(npix.max())
    dev = torch.device("cuda:0")
    up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    data, sizes, offs, init = up(batch.data), up(batch.sizes), up(batch.offsets), up(batch.init)
    ctx = sf.Context(0)
    prec = {"fp64": sf.PREC_FP64, "mixed": sf.PREC_MIXED, "fp32": sf.PREC_FP32,
            "plain": sf.PREC_FP32_PLAIN, "comp": sf.PREC_COMP}[a.precision]
    max_side = int(max(batch.sizes[:, 0].max(), batch.sizes[:, 1].max()))
    opts = sf.default_options(precision=prec, max_pixels=max(9, max_px), max_side=max(3, max_side),
                              tie_tau=a.tie_tau,
                              schedule=sf.SCHEDULE_MIXED if a.schedule == "mixed" else sf.SCHEDULE_UNIFORM)
    if a.schedule == "mixed":
        ctx.reserve(n)
    out = ctx.fit_spots(data, sizes, offs, init, opts, want_evals=True)
    torch.cuda.synchronize()

    # per-size launches: the spots of each ROI side as their own batch, in device
    # memory before timing; one step launches them all
    groups = []
    if a.schedule == "per-size":
        side_of = np.maximum(batch.sizes[:, 0], batch.sizes[:, 1])
        for side in np.unique(side_of):
            idx = np.nonzero(side_of == side)[0]
            sub = batch.subset(idx)
            o2 = sf.default_options(precision=prec, max_pixels=max(9, int(sub.npix().max())),
                                    max_side=int(max(3, side)), tie_tau=a.tie_tau)
            groups.append((idx, o2, up(sub.data), up(sub.sizes), up(sub.offsets), up(sub.init),
                           ctx.fit_spots(up(sub.data), up(sub.sizes), up(sub.offsets),
                                         up(sub.init), o2)))
        torch.cuda.synchronize()

    def step(stream):
        if groups:
            for idx, o2, d, sz, of, it, ou in groups:
                ctx.fit_spots(d, sz, of, it, o2, out=ou, stream=stream)
        else:
            ctx.fit_spots(data, sizes, offs, init, opts, out=out, stream=stream)

    # algorithmic work from the evaluation counts (the fit is deterministic, so the
    # timed launches below do exactly this work)
    ev = out["evals"].cpu().numpy().astype(np.int64)
    models = batch.sizes[:, 2].astype(np.int64)
    cg = np.where(models == 1, C_GRAD[1], C_GRAD[0])
    ng, nt = ev[:, 0], ev[:, 1]
    flops = float((npix * (cg * ng + C_TRIAL * nt - 11 * np.maximum(ng - 1, 0))).sum())
    exps = float((npix * (nt + 1)).sum())
    bytes_in = float(batch.data.nbytes + batch.sizes.nbytes + batch.offsets.nbytes +
                     batch.init.nbytes)
    bytes_out = float(n * (6 * 4 + 4 + 4 + 4))
    alg_bytes = bytes_in + bytes_out
    status = out["status"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    del out["evals"]

    stream = torch.cuda.current_stream(dev)
    for _ in range(a.warmup):
        step(stream)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(a.steps):
        starts[i].record(stream)
        step(stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    k_avg_s = sum(kms) / len(kms) / 1e3
    ms_per_step = wall / a.steps * 1e3
    fits_per_s = n / (wall / a.steps)

    if a.pmc_copy_mb > 0:
        src = torch.ones(a.pmc_copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    achieved_tflops = flops / k_avg_s / 1e12
    hbm_gbps = alg_bytes / k_avg_s / 1e9
    traffic = measured_traffic(a.workload, a.precision, a.schedule)

    # end to end (outside the timed region): pinned host inputs -> device, the fit,
    # the results -> pinned host memory, one synchronisation per call
    e2e = None
    if a.e2e_reps > 0 and not groups:
        h_in = [torch.from_numpy(np.ascontiguousarray(x)).pin_memory()
                for x in (batch.data, batch.sizes, batch.offsets, batch.init)]
        d_in = [torch.empty_like(x, device=dev) for x in h_in]
        h_out = {k: torch.empty(v.shape, dtype=v.dtype).pin_memory() for k, v in out.items()}

        def e2e_call():
            for h, d in zip(h_in, d_in):
                d.copy_(h, non_blocking=True)
            ctx.fit_spots(*d_in, opts, out=out, stream=stream)
            for k, v in out.items():
                h_out[k].copy_(v, non_blocking=True)
            torch.cuda.synchronize()

        e2e_call()
        t0 = time.perf_counter()
        for _ in range(a.e2e_reps):
            e2e_call()
        e_s = (time.perf_counter() - t0) / a.e2e_reps
        in_bytes = sum(x.numel() * x.element_size() for x in h_in)
        out_bytes = sum(v.numel() * v.element_size() for v in h_out.values())
        e2e = {"fits_per_s": n / e_s, "ms_per_call": e_s * 1e3, "reps": a.e2e_reps,
               "host_to_device_bytes": in_bytes, "device_to_host_bytes": out_bytes}
        del h_in, d_in, h_out

    # serving: frames with Poisson arrivals through the serving loop (outside the
    # timed region; its own clock is per frame, arrival -> results on the host)
    serve = None
    if a.serve_frames > 0:
        from paper_2106_02045_amd import serve_bench
        sv = serve_bench.run(["--frames", str(a.serve_frames), "--fps", str(a.serve_fps),
                              "--streams", "2", "--check", "20"])
        serve = {"workload": "serve_fiducials", "frames": sv["frames"],
                 "fps_offered": sv["fps_offered"], "fps_achieved": sv["fps_achieved"],
                 "p50_us": sv["latency_p50_us"], "p99_us": sv["latency_p99_us"],
                 "max_us": sv["latency_max_us"], "fits_per_s": sv["fits_per_s"],
                 "frames_per_launch": sv["mean_frames_per_batch"], "plan": sv["plan"],
                 "warmup_frames": sv["warmup_frames"],
                 "alone_vs_mix_differing": sv["alone_vs_mix"]["frames_differing"]}

    # issue utilisation from the hardware counters of one launch of this kernel
    # build (committed summary, stamped with the sources' hash): VALU wave
    # instructions x 4 cycles over the SIMD cycles of the measured launch time
    valu = None
    cnt = measured_counters(a.workload, a.precision, a.schedule)
    if cnt is not None:
        simd_cycles = 256 * 4 * CLOCK_HZ * k_avg_s
        f64 = cnt["SQ_INSTS_VALU_FMA_F64"] * 2 + cnt["SQ_INSTS_VALU_MUL_F64"] + \
            cnt["SQ_INSTS_VALU_ADD_F64"]
        valu = {"issue_frac": cnt["SQ_INSTS_VALU"] * 4 / simd_cycles,
                "fp64_flop_frac": f64 * 64 / k_avg_s / (PEAK_ALU_TFLOPS * 1e12),
                "valu_insts_per_launch": cnt["SQ_INSTS_VALU"],
                "fp64_flops_per_launch": f64 * 64,
                "busy_frac_counters": cnt.get("valu_busy_frac"),
                "source": os.path.join("profiles", os.path.basename(cnt["_path"]))
                if "_path" in cnt else None}

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        m = min(a.cpu_sample, n)
        sub = spotgen.workload(a.workload, n=m)
        hc = host_cpu()
        # at most 16 threads: the share of the host's cores that one GPU's jobs may use
        threads = a.cpu_threads or min(hc["allowed"] or hc["nproc"] or 1, 16)
        lib, flags = oracle.native_lib()
        oo = oracle.default_opts(tie_tau=a.tie_tau)
        c0 = time.perf_counter()
        oracle.fit_batch(sub, oo, threads=threads, library=lib)
        cs = time.perf_counter() - c0
        cpu = {"value": m / cs, "unit": "fits/s", "cores": threads, "kind": "oracle",
               "sample": f"first {m} spots of {a.workload} (same generator and seed), "
                         f"{cs:.2f} s wall on {threads} threads",
               "host": hc, "build": flags}
        if a.cpu_sample_1t > 0:
            m1 = min(a.cpu_sample_1t, n)
            sub1 = sub.subset(np.arange(m1)) if m1 < m else sub
            c0 = time.perf_counter()
            oracle.fit_batch(sub1, oo, threads=1, library=lib)
            c1 = time.perf_counter() - c0
            cpu["single_thread"] = {"value": m1 / c1, "unit": "fits/s", "cores": 1,
                                    "sample": f"first {m1} spots of {a.workload}, {c1:.2f} s wall"}

    parity = None
    if a.parity_sample > 0:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import compare
        rng = np.random.default_rng(12345)
        idx = np.sort(rng.choice(n, size=min(a.parity_sample, n), replace=False))
        r = oracle.fit_batch(batch.subset(idx), oracle.default_opts(tie_tau=a.tie_tau),
                             threads=min(os.cpu_count() or 1, 16))
        full = {k: out[k].cpu().numpy() for k in ("params", "chi2", "iters", "status")}
        for gidx, o2, d, sz, of, it, ou in groups:  # per-size results back in spot order
            for k in full:
                full[k][gidx] = ou[k].cpu().numpy()
        g = {k: v[idx] for k, v in full.items()}
        c = compare(g, r, chi_band=1e-11, step_band=1e-9)
        parity = {"sample": len(idx), "status_mismatch": c["status_mismatch"],
                  "iters_mismatch": c["iters_mismatch"], "tol_fail": c["tol_fail_any"],
                  "max_abs_dxy_px": c["max_dxy"], "max_rel_sigma_alpha_beta": c["max_rel"],
                  "max_rel_chi2": c["max_rchi"], "median_rel_chi2": c["med_rchi"]}

    rec = {
        "metric": "fits/s",
        "value": fits_per_s,
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {sf.PREC_FP64: "f64", sf.PREC_MIXED: "f32+f64", sf.PREC_FP32: "f32",
                  sf.PREC_FP32_PLAIN: "f32", sf.PREC_COMP: "f32 compensated+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": a.workload, "spots": n, "roi": f"{batch.sizes[0,0]}x{batch.sizes[0,1]}"
                   if len(np.unique(npix)) == 1 else "mixed", "pixel_dtype": "u16",
                   "precision": a.precision, "tie_tau": a.tie_tau, "schedule": a.schedule,
                   "launches_per_step": max(1, len(groups))},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_ALU_TFLOPS,
                     "traffic": traffic},
        "hbm": {"achieved_algorithmic_GBps": hbm_gbps, "peak_GBps": PEAK_HBM_GBPS,
                "frac": hbm_gbps / PEAK_HBM_GBPS, "bytes_per_launch": alg_bytes,
                "measured_GBps": traffic / k_avg_s / 1e9 if traffic is not None else None},
        "end_to_end": e2e,
        "kernel_ms_avg": k_avg_s * 1e3,
        "exp_per_s": exps / k_avg_s,
        "evals_per_spot": {"grad": float(ng.mean()), "trial": float(nt.mean())},
        "status_hist": np.bincount(status, minlength=6).tolist(),
        "iters_mean": float(iters.mean()),
        "valu": valu,
        "serve": serve,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "gen_s": gen_s,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
