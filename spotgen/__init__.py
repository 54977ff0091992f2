"""Seeded synthetic spot images: the inputs shared by the FP64 oracle and the HIP path.

This module holds no arithmetic of the fitting method itself.  It draws spot
parameters, renders noisy images of them, and prepares initial shaping
parameters with a simple moment estimator, exactly as a camera pipeline
upstream of the fitter would.  Both the oracle and the GPU path take its
outputs as plain inputs.

Data layout handed to both sides (the same layout the C-ABI takes):
  data     uint16 (or float32) flat array, spot s occupies
           data[offsets[s] : offsets[s] + w*h], row-major (pixel k = row*w + col)
  sizes    uint8 [n, 4] = (w, h, model, 0); model 0 = symmetric, 1 = elliptical
  offsets  int64 [n] element offsets into data
  init     float32 [n, 4] = (x, y, sigma_x, sigma_y); symmetric spots use sigma_x
  truth    float64 [n, 6] = (x, y, sigma_x, sigma_y, alpha, beta) used to render

Coordinates are 0-based pixel centres: x is the column, y the row.

Randomness: numpy PCG64.  Spots are generated in fixed chunks of CHUNK spots;
chunk c uses the stream SeedSequence([seed, c]) and draws, in this order:
side, model, centre offset, sigma(s), amplitude, background, then the pixel
noise of the whole chunk.  A prefix of a large configuration is therefore
identical to the smaller configuration with the same seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

CHUNK = 4096
SYM, ELL = 0, 1
MAX_PIXELS = 1024


@dataclasses.dataclass
class SpotBatch:
    data: np.ndarray
    sizes: np.ndarray
    offsets: np.ndarray
    init: np.ndarray
    truth: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.sizes.shape[0])

    def npix(self) -> np.ndarray:
        return self.sizes[:, 0].astype(np.int64) * self.sizes[:, 1].astype(np.int64)

    def spot(self, s: int) -> np.ndarray:
        w, h = int(self.sizes[s, 0]), int(self.sizes[s, 1])
        o = int(self.offsets[s])
        return self.data[o:o + w * h].reshape(h, w)

    def subset(self, idx) -> "SpotBatch":
        """Repack the chosen spots into a new contiguous batch."""
        idx = np.asarray(idx, dtype=np.int64)
        npx = self.npix()[idx]
        offs = np.zeros(len(idx), dtype=np.int64)
        if len(idx):
            offs[1:] = np.cumsum(npx)[:-1]
        data = np.empty(int(npx.sum()), dtype=self.data.dtype)
        for j, s in enumerate(idx):
            o = int(self.offsets[s])
            data[offs[j]:offs[j] + npx[j]] = self.data[o:o + npx[j]]
        return SpotBatch(data, self.sizes[idx].copy(), offs, self.init[idx].copy(),
                         self.truth[idx].copy(), self.name + "[subset]")


# ----------------------------------------------------------------------------
# Laws of the named workloads.  Each returns per-spot arrays for one chunk.
# ----------------------------------------------------------------------------

def _law_small(rng, m):
    # 11x11 symmetric, sigma U[1.2,2], centre +-1 px, alpha U[500,2000], beta 100, Poisson.
    side = np.full(m, 11)
    model = np.full(m, SYM)
    off = rng.uniform(-1.0, 1.0, size=(m, 2))
    s = rng.uniform(1.2, 2.0, size=m)
    sig = np.stack([s, s], 1)
    alpha = rng.uniform(500.0, 2000.0, size=m)
    beta = np.full(m, 100.0)
    return side, side, model, off, sig, alpha, beta, 0.0


def _law_scale(rng, m):
    # 15x15 symmetric, sigma U[1,3], alpha log-uniform [1e2,1e4], beta U[10,200],
    # Poisson plus Gaussian read noise of sd 2 counts.
    side = np.full(m, 15)
    model = np.full(m, SYM)
    off = rng.uniform(-1.0, 1.0, size=(m, 2))
    s = rng.uniform(1.0, 3.0, size=m)
    sig = np.stack([s, s], 1)
    alpha = 10.0 ** rng.uniform(2.0, 4.0, size=m)
    beta = rng.uniform(10.0, 200.0, size=m)
    return side, side, model, off, sig, alpha, beta, 2.0


def _law_precision(rng, m):
    # 32x32 elliptical, sigma_x, sigma_y U[1.5,6], alpha U[50,300], beta U[200,1000], Poisson.
    side = np.full(m, 32)
    model = np.full(m, ELL)
    off = rng.uniform(-1.0, 1.0, size=(m, 2))
    sig = rng.uniform(1.5, 6.0, size=(m, 2))
    alpha = rng.uniform(50.0, 300.0, size=m)
    beta = rng.uniform(200.0, 1000.0, size=m)
    return side, side, model, off, sig, alpha, beta, 0.0


MIXED_SIDES = np.array([7, 9, 11, 15, 21, 25, 32])


def _law_mixed(rng, m):
    # side U{7,9,11,15,21,25,32}; half symmetric, half elliptical; sigma U[1,3]
    # per axis; amplitude, background and noise laws of the 15x15 workload
    # (alpha log-uniform [1e2,1e4], beta U[10,200], Poisson plus read noise sd 2).
    side = MIXED_SIDES[rng.integers(0, len(MIXED_SIDES), size=m)]
    model = rng.integers(0, 2, size=m)
    off = rng.uniform(-1.0, 1.0, size=(m, 2))
    sig = rng.uniform(1.0, 3.0, size=(m, 2))
    sig[model == SYM, 1] = sig[model == SYM, 0]
    alpha = 10.0 ** rng.uniform(2.0, 4.0, size=m)
    beta = rng.uniform(10.0, 200.0, size=m)
    return side, side, model, off, sig, alpha, beta, 2.0


def _law_mixed_low(rng, m):
    # the mixed sizes and models with the low-contrast laws of the 32x32 workload
    # (alpha U[50,300], beta U[200,1000], Poisson): dim spots whose trials are
    # often worse, for tests of the damping retries and their cap.
    side = MIXED_SIDES[rng.integers(0, len(MIXED_SIDES), size=m)]
    model = rng.integers(0, 2, size=m)
    off = rng.uniform(-1.0, 1.0, size=(m, 2))
    sig = rng.uniform(1.0, 3.0, size=(m, 2))
    sig[model == SYM, 1] = sig[model == SYM, 0]
    alpha = rng.uniform(50.0, 300.0, size=m)
    beta = rng.uniform(200.0, 1000.0, size=m)
    return side, side, model, off, sig, alpha, beta, 0.0


SERVE_SIDES = np.array([9, 13, 17, 21])


def _law_serve(rng, m):
    # fiducial spots of the camera-frame stream: side in {9,13,17,21}, symmetric,
    # sigma U[1.5,2.5], alpha U[1000,5000], beta 150, Poisson.
    side = SERVE_SIDES[rng.integers(0, len(SERVE_SIDES), size=m)]
    model = np.full(m, SYM)
    off = rng.uniform(-1.0, 1.0, size=(m, 2))
    s = rng.uniform(1.5, 2.5, size=m)
    sig = np.stack([s, s], 1)
    alpha = rng.uniform(1000.0, 5000.0, size=m)
    beta = np.full(m, 150.0)
    return side, side, model, off, sig, alpha, beta, 0.0


WORKLOADS = {
    # name: (law, default count, default seed)
    "small_11x11": (_law_small, 1024, 0),
    "scale_15x15": (_law_scale, 1_000_000, 1),
    "precision_32x32_ell": (_law_precision, 1_000_000, 2),
    "mixed_7to32": (_law_mixed, 2_000_000, 3),
    "serve_fiducials": (_law_serve, 0, 4),
    "mixed_low_contrast": (_law_mixed_low, 20000, 5),
}
CONFIG_NAMES = ["small_11x11", "scale_15x15", "precision_32x32_ell", "mixed_7to32",
                "serve_fiducials"]


# ----------------------------------------------------------------------------
# Rendering and the moment initialiser
# ----------------------------------------------------------------------------

def _render_group(w, h, cx, cy, sx, sy, alpha, beta):
    """Noise-free expected counts, point-sampled at pixel centres. shape (m, h*w)."""
    xs = np.arange(w, dtype=np.float64)
    ys = np.arange(h, dtype=np.float64)
    ex = np.exp(-0.5 * ((xs[None, :] - cx[:, None]) / sx[:, None]) ** 2)  # (m, w)
    ey = np.exp(-0.5 * ((ys[None, :] - cy[:, None]) / sy[:, None]) ** 2)  # (m, h)
    prof = ey[:, :, None] * ex[:, None, :]
    lam = alpha[:, None, None] * prof + beta[:, None, None]
    return lam.reshape(len(cx), h * w)


def moment_init(img: np.ndarray, model: int) -> np.ndarray:
    """Centroid / second-moment start values for a stack of equal-size images.

    img: (m, h, w) float64.  Background b0 = median of the border ring; weights
    w = max(g - b0, 0); centre = weighted centroid; symmetric sigma^2 =
    sum w r^2 / (2 sum w), elliptical sigma_x^2 = sum w dx^2 / sum w (same for y).
    Sigma is kept in [0.8, max(w, h)/4]; an image with no positive weight starts
    at the ROI centre with sigma 1.5.  Returns float64 (m, 4).
    """
    m, h, w = img.shape
    ring = np.concatenate([img[:, 0, :], img[:, -1, :], img[:, 1:-1, 0], img[:, 1:-1, -1]], axis=1)
    b0 = np.median(ring, axis=1)
    wt = np.maximum(img - b0[:, None, None], 0.0)
    sw = wt.sum(axis=(1, 2))
    ok = sw > 0
    swd = np.where(ok, sw, 1.0)
    xs = np.arange(w, dtype=np.float64)[None, None, :]
    ys = np.arange(h, dtype=np.float64)[None, :, None]
    cx = (wt * xs).sum(axis=(1, 2)) / swd
    cy = (wt * ys).sum(axis=(1, 2)) / swd
    dx2 = (wt * (xs - cx[:, None, None]) ** 2).sum(axis=(1, 2)) / swd
    dy2 = (wt * (ys - cy[:, None, None]) ** 2).sum(axis=(1, 2)) / swd
    if model == SYM:
        s = np.sqrt(0.5 * (dx2 + dy2))
        sx = sy = s
    else:
        sx, sy = np.sqrt(dx2), np.sqrt(dy2)
    lo, hi = 0.8, max(w, h) / 4.0
    sx = np.clip(sx, lo, hi)
    sy = np.clip(sy, lo, hi)
    out = np.stack([cx, cy, sx, sy], axis=1)
    out[~ok] = [(w - 1) / 2.0, (h - 1) / 2.0, 1.5, 1.5]
    return out


def paper_init(img: np.ndarray) -> np.ndarray:
    """The initial-value recipe the paper describes for its accuracy runs.

    3x3 moving average (mean over the in-bounds part of the window); centre at the
    brightest smoothed pixel; beta0 = lowest pixel, alpha0 = highest pixel - beta0;
    sigma = sqrt(M / pi) with M the number of raw pixels above alpha0*exp(-1/2)+beta0.
    img: (m, h, w).  Returns float64 (m, 4) = (x, y, sigma, sigma); sigma >= 0.5.
    """
    m, h, w = img.shape
    pad = np.pad(img, ((0, 0), (1, 1), (1, 1)))
    cnt = np.pad(np.ones((h, w)), 1)
    acc = np.zeros_like(img)
    nacc = np.zeros((h, w))
    for dy in range(3):
        for dx in range(3):
            acc += pad[:, dy:dy + h, dx:dx + w]
            nacc += cnt[dy:dy + h, dx:dx + w]
    sm = acc / nacc[None]
    k = sm.reshape(m, -1).argmax(axis=1)
    y0, x0 = np.divmod(k, w)
    b0 = img.reshape(m, -1).min(axis=1)
    a0 = img.reshape(m, -1).max(axis=1) - b0
    thr = a0 * math.exp(-0.5) + b0
    M = (img.reshape(m, -1) > thr[:, None]).sum(axis=1)
    s = np.maximum(np.sqrt(M / math.pi), 0.5)
    return np.stack([x0.astype(np.float64), y0.astype(np.float64), s, s], axis=1)


def _finish_chunk(rng, side_w, side_h, model, off, sig, alpha, beta, read_sd, dtype,
                  init_fn: Callable[[np.ndarray, int], np.ndarray], noise: str = "poisson"):
    m = len(side_w)
    cx = (side_w - 1) / 2.0 + off[:, 0]
    cy = (side_h - 1) / 2.0 + off[:, 1]
    npx = (side_w * side_h).astype(np.int64)
    offs = np.zeros(m, dtype=np.int64)
    offs[1:] = np.cumsum(npx)[:-1]
    lam = np.empty(int(npx.sum()), dtype=np.float64)
    keys = side_w.astype(np.int64) * 4096 + side_h.astype(np.int64) * 2 + model.astype(np.int64)
    groups = {}
    for key in np.unique(keys):
        idx = np.nonzero(keys == key)[0]
        w, h = int(side_w[idx[0]]), int(side_h[idx[0]])
        groups[key] = (idx, w, h)
        L = _render_group(w, h, cx[idx], cy[idx], sig[idx, 0], sig[idx, 1], alpha[idx], beta[idx])
        pos = offs[idx][:, None] + np.arange(w * h)[None, :]
        lam[pos] = L
    if noise == "poisson":
        g = rng.poisson(lam).astype(np.float64)
        if read_sd > 0:
            g += rng.normal(0.0, read_sd, size=g.shape)
    elif noise == "gauss_var":
        g = lam + rng.normal(0.0, 1.0, size=lam.shape) * np.sqrt(lam)
    elif noise == "none":
        g = lam.copy()
    else:
        raise ValueError(noise)
    if dtype == np.uint16:
        g = np.clip(np.rint(g), 0, 65535)
    data = g.astype(dtype)
    init = np.empty((m, 4), dtype=np.float64)
    for key, (idx, w, h) in groups.items():
        pos = offs[idx][:, None] + np.arange(w * h)[None, :]
        img = data[pos].astype(np.float64).reshape(len(idx), h, w)
        init[idx] = init_fn(img, int(model[idx[0]]))
    sizes = np.zeros((m, 4), dtype=np.uint8)
    sizes[:, 0] = side_w
    sizes[:, 1] = side_h
    sizes[:, 2] = model
    truth = np.stack([cx, cy, sig[:, 0], sig[:, 1], alpha, beta], axis=1)
    return data, sizes, offs, init.astype(np.float32), truth


def _concat(parts, name):
    datas, sizes, offs, inits, truths = zip(*parts)
    base = 0
    offs2 = []
    for d, o in zip(datas, offs):
        offs2.append(o + base)
        base += len(d)
    return SpotBatch(np.concatenate(datas), np.concatenate(sizes), np.concatenate(offs2),
                     np.concatenate(inits), np.concatenate(truths), name)


def workload(name: str, n: Optional[int] = None, seed: Optional[int] = None,
             dtype=np.uint16, noise: str = "poisson", threads: int = 1) -> SpotBatch:
    """Generate the first n spots of a named workload (see WORKLOADS)."""
    law, n_def, seed_def = WORKLOADS[name]
    n = n_def if n is None else int(n)
    seed = seed_def if seed is None else int(seed)
    nchunks = (n + CHUNK - 1) // CHUNK

    def one(c):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c])))
        m = min(CHUNK, n - c * CHUNK)
        side_w, side_h, model, off, sig, alpha, beta, rsd = law(rng, CHUNK)
        # always render the whole chunk so that every draw sits at the same stream
        # position whatever n is, then keep the first m spots
        d, sz, of, ini, tr = _finish_chunk(rng, side_w, side_h, model, off, sig, alpha, beta, rsd,
                                           dtype, moment_init, noise)
        end = int(of[m]) if m < CHUNK else len(d)
        return d[:end], sz[:m], of[:m], ini[:m], tr[:m]

    if nchunks == 0:
        return SpotBatch(np.zeros(0, dtype), np.zeros((0, 4), np.uint8), np.zeros(0, np.int64),
                         np.zeros((0, 4), np.float32), np.zeros((0, 6)), name)
    if threads > 1 and nchunks > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(one, range(nchunks)))
    else:
        parts = [one(c) for c in range(nchunks)]
    return _concat(parts, name)


def config(i: int, n: Optional[int] = None, **kw) -> SpotBatch:
    return workload(CONFIG_NAMES[i], n=n, **kw)


def paper_protocol(n: int, S: int, n_signal: float, n_background: float, seed: int = 7,
                   init: str = "paper") -> SpotBatch:
    """The paper's simulated accuracy workload (Results section).

    S x S ROI; centre normal around the ROI centre with sd S/20; sigma U[1,2];
    peak alpha from the integrated signal, alpha = N_signal / (2 pi sigma^2);
    background N_background / S^2 per pixel; Gaussian noise of variance equal to
    the expected intensity; rounded to non-negative integers.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, S, int(n_signal),
                                                                        int(n_background)])))
    side = np.full(n, S)
    model = np.full(n, SYM)
    off = rng.normal(0.0, S / 20.0, size=(n, 2))
    s = rng.uniform(1.0, 2.0, size=n)
    sig = np.stack([s, s], 1)
    alpha = n_signal / (2.0 * math.pi * s * s)
    beta = np.full(n, n_background / (S * S))
    init_fn = (lambda img, mdl: paper_init(img)) if init == "paper" else moment_init
    parts = _finish_chunk(rng, side, side, model, off, sig, alpha, beta, 0.0, np.uint16, init_fn,
                          noise="gauss_var")
    return _concat([parts], f"paper_{S}x{S}_{n_signal:g}_{n_background:g}")


def noise_free(n: int, sides=(9, 11, 15), models=(SYM, ELL), seed: int = 11) -> SpotBatch:
    """Noise-free float32 spots (exact renders) with a moment init, for recovery tests."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 99])))
    side = np.asarray(sides)[rng.integers(0, len(sides), size=n)]
    model = np.asarray(models)[rng.integers(0, len(models), size=n)]
    off = rng.uniform(-1.0, 1.0, size=(n, 2))
    sig = rng.uniform(1.2, 2.5, size=(n, 2))
    sig[model == SYM, 1] = sig[model == SYM, 0]
    alpha = rng.uniform(200.0, 3000.0, size=n)
    beta = rng.uniform(10.0, 300.0, size=n)
    parts = _finish_chunk(rng, side, side, model, off, sig, alpha, beta, 0.0, np.float32,
                          moment_init, noise="none")
    return _concat([parts], "noise_free")


def serve_frames(n_frames: int, fps: float = 1000.0, seed: int = 4,
                 spots_lo: int = 20, spots_hi: int = 200, pool_spots: int = 200000,
                 threads: int = 1):
    """Camera-frame stream: Poisson arrivals at `fps`, U{spots_lo..spots_hi} spots each.

    Returns (arrival times in seconds, list of per-frame SpotBatch).  Spots come from
    one seeded pool of the serve_fiducials law; frame f takes the next counts[f]
    spots of the pool, cycling through it (a stream longer than the pool reuses
    spots, which leaves the per-frame size and work distribution unchanged).
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 4242])))
    gaps = rng.exponential(1.0 / fps, size=n_frames)
    t = np.cumsum(gaps)
    counts = rng.integers(spots_lo, spots_hi + 1, size=n_frames)
    total = int(counts.sum())
    pool = workload("serve_fiducials", n=max(spots_hi, min(total, pool_spots)), seed=seed,
                    threads=threads)
    npix = pool.npix()
    frames = []
    cur = 0
    for f in range(n_frames):
        c = int(counts[f])
        if cur + c > pool.n:
            cur = 0
        s0, s1 = cur, cur + c
        cur = s1
        o0 = int(pool.offsets[s0])
        o1 = o0 + int(npix[s0:s1].sum())
        frames.append(SpotBatch(pool.data[o0:o1], pool.sizes[s0:s1], pool.offsets[s0:s1] - o0,
                                pool.init[s0:s1], pool.truth[s0:s1], f"frame{f}"))
    return t, frames


def drift_frames(n_frames: int, n_markers: int = 32, side: int = 13, fps: float = 1000.0,
                 seed: int = 6, walk_sd: float = 0.002, sway: float = 0.3,
                 sway_period_s: float = 2.0):
    """Frames of fixed fiducial markers whose sample drifts (the tracking workload).

    Each marker has its own ROI (side x side), sub-ROI position (centre +- 1 px),
    sigma U[1.5, 2.5], peak U[1000, 5000] and background 150.  The sample moves
    every marker by the same drift d(f) = random walk (step sd walk_sd px per
    frame) + a sway of amplitude `sway` px and period sway_period_s at `fps`.
    Pixels are point-sampled, Poisson noise, uint16.  Returns (ref [M, 2] true
    marker positions at zero drift, drift [F, 2] true drift per frame, list of
    per-frame SpotBatch with the markers in order and moment start values).
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 5151])))
    M = int(n_markers)
    c0 = (side - 1) / 2.0
    ref = c0 + rng.uniform(-1.0, 1.0, size=(M, 2))
    sig = rng.uniform(1.5, 2.5, size=M)
    alpha = rng.uniform(1000.0, 5000.0, size=M)
    beta = np.full(M, 150.0)
    steps = rng.normal(0.0, walk_sd, size=(n_frames, 2))
    walk = np.cumsum(steps, axis=0)
    ph = 2.0 * math.pi * np.arange(n_frames) / (fps * sway_period_s)
    drift = walk + sway * np.stack([np.sin(ph), 0.5 * np.sin(2.0 * ph + 1.0)], axis=1)
    frames = []
    sizes = np.zeros((M, 4), dtype=np.uint8)
    sizes[:, 0] = sizes[:, 1] = side
    offs = np.arange(M, dtype=np.int64) * side * side
    for f in range(n_frames):
        cx = ref[:, 0] + drift[f, 0]
        cy = ref[:, 1] + drift[f, 1]
        lam = _render_group(side, side, cx, cy, sig, sig, alpha, beta).reshape(-1)
        g = np.clip(np.rint(rng.poisson(lam).astype(np.float64)), 0, 65535)
        data = g.astype(np.uint16)
        init = moment_init(data.astype(np.float64).reshape(M, side, side), SYM).astype(np.float32)
        truth = np.stack([cx, cy, sig, sig, alpha, beta], axis=1)
        frames.append(SpotBatch(data, sizes.copy(), offs.copy(), init, truth, f"drift{f}"))
    return ref, drift, frames
