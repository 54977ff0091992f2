"""TEST INFRASTRUCTURE ONLY: ctypes binding of the double-precision CPU oracle.

The oracle (spotfit_oracle.c, plain serial C in double precision) is the
reference the HIP path is checked against.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this module; the product
package never does.  It shares no code with the HIP path.

Parity status: see the header of spotfit_oracle.h (what pins each function).
drift_track (the drift-tracking consumer of fitted marker positions) is plain
numpy here, pinned by exact shifts, excluded markers and a linear drift.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "spotfit_oracle.c")

MAX_ITER, MAX_ERROR, MIN_DELTA, MIN_STEP, NOT_CONVERGED, BAD_INPUT = range(6)
STATUS_NAMES = ["MAX_ITER", "MAX_ERROR", "MIN_DELTA", "MIN_STEP", "NOT_CONVERGED", "BAD_INPUT"]


class Opts(ctypes.Structure):
    _fields_ = [
        ("max_iter", ctypes.c_int32),
        ("max_error_per_px", ctypes.c_double),
        ("min_delta", ctypes.c_double),
        ("min_step_rel", ctypes.c_double),
        ("lambda0_exp10", ctypes.c_int32),
        ("lambda_max_exp10", ctypes.c_int32),
        ("tie_tau", ctypes.c_double),
        ("sigma_min", ctypes.c_double),
        ("sigma_max_frac", ctypes.c_double),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("params", ctypes.c_double * 6),
        ("chi2", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("n_grad", ctypes.c_int32),
        ("n_trial", ctypes.c_int32),
        ("margin_chi", ctypes.c_double),
        ("margin_step", ctypes.c_double),
        ("min_pivot", ctypes.c_double),
    ]


class Event(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("iter", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("p", ctypes.c_double * 4),
        ("delta", ctypes.c_double * 4),
        ("chi", ctypes.c_double),
    ]


EV_GRAD, EV_TRIAL, EV_RETRY = range(3)


# the build the tests load (and that travels with the tree): baseline x86-64
PORTABLE_FLAGS = ["-O3", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc: baseline x86-64, no fast-math, no FMA contraction."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", *PORTABLE_FLAGS, "-fPIC", "-shared", "-std=gnu99", "-Wall", "-o",
                        tmp, SRC_PATH, "-lm", "-lpthread"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = bind(ctypes.CDLL(LIB_PATH))
    return _lib


def bind(L):
    """Declare the argument and return types of the oracle's functions on a loaded
    library (this one, or a copy built from edited sources by a test)."""
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.orc_eval.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                           dp, dp, dp, dp]
    L.orc_eval.restype = ctypes.c_int
    L.orc_solve.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, dp]
    L.orc_solve.restype = ctypes.c_int
    L.orc_pow10.argtypes = [ctypes.c_int]
    L.orc_pow10.restype = ctypes.c_double
    L.orc_fit_spot.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_float), ctypes.POINTER(Opts),
                               ctypes.POINTER(Result)]
    L.orc_fit_spot_traced.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_float), ctypes.POINTER(Opts),
                                      ctypes.POINTER(Result), ctypes.POINTER(Event),
                                      ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    vp = ctypes.c_void_p
    L.orc_fit_batch.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_int64,
                                ctypes.POINTER(Opts), vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                ctypes.c_int]
    L.orc_fit_batch.restype = ctypes.c_int
    L.orc_moment_init.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
    L.orc_moment_init.restype = ctypes.c_int
    L.orc_moment_init_batch.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int64, vp]
    L.orc_moment_init_batch.restype = ctypes.c_int
    L.orc_peak_init.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
    L.orc_peak_init.restype = ctypes.c_int
    L.orc_peak_init_batch.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int64, vp]
    L.orc_peak_init_batch.restype = ctypes.c_int
    return L


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().orc_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def nparams(model: int) -> int:
    return 3 if model == 0 else 4


def eval_spot(g, w: int, h: int, model: int, p, grad: bool = True, want_J: bool = False):
    """One model evaluation.  Returns dict(alpha, beta, chi2, A, b, J, rc)."""
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
    assert g.size == w * h
    n = nparams(model)
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64)[:n])
    out3 = np.zeros(3)
    A = np.zeros((n, n))
    b = np.zeros(n)
    J = np.zeros((w * h, n)) if want_J else None
    rc = lib().orc_eval(_dp(g), w, h, model, _dp(p), int(grad), _dp(out3), _dp(A), _dp(b),
                        _dp(J) if J is not None else None)
    return dict(alpha=out3[0], beta=out3[1], chi2=out3[2], A=A, b=b, J=J, rc=rc)


def solve(A, b, lam: float):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    d = np.zeros(len(b))
    rc = lib().orc_solve(_dp(A), _dp(b), len(b), float(lam), _dp(d))
    return d, rc


def pow10(k: int) -> float:
    return lib().orc_pow10(int(k))


def fit_spot(g, w: int, h: int, model: int, init4, opts: Optional[Opts] = None) -> dict:
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
    init4 = np.ascontiguousarray(np.asarray(init4, dtype=np.float32).reshape(4))
    o = opts if opts is not None else default_opts()
    r = Result()
    lib().orc_fit_spot(_dp(g), w, h, model, init4.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                       ctypes.byref(o), ctypes.byref(r))
    return dict(params=np.array(r.params[:]), chi2=r.chi2, iters=r.iters, status=r.status,
                n_grad=r.n_grad, n_trial=r.n_trial, margin_chi=r.margin_chi,
                margin_step=r.margin_step, min_pivot=r.min_pivot)


def fit_spot_traced(g, w: int, h: int, model: int, init4, opts: Optional[Opts] = None,
                    cap: int = 2048):
    """fit_spot plus the loop's trajectory: (result dict, list of event dicts with
    kind (EV_GRAD / EV_TRIAL / EV_RETRY), iter, k, p, delta, chi)."""
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
    init4 = np.ascontiguousarray(np.asarray(init4, dtype=np.float32).reshape(4))
    o = opts if opts is not None else default_opts()
    r = Result()
    ev = (Event * cap)()
    n_ev = ctypes.c_int(0)
    lib().orc_fit_spot_traced(_dp(g), w, h, model,
                              init4.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                              ctypes.byref(o), ctypes.byref(r), ev, cap, ctypes.byref(n_ev))
    if n_ev.value > cap:
        raise RuntimeError(f"trajectory of {n_ev.value} events exceeds cap {cap}")
    n = nparams(model)
    events = [dict(kind=e.kind, iter=e.iter, k=e.k, p=np.array(e.p[:n]),
                   delta=np.array(e.delta[:n]), chi=e.chi) for e in ev[:n_ev.value]]
    res = dict(params=np.array(r.params[:]), chi2=r.chi2, iters=r.iters, status=r.status,
               n_grad=r.n_grad, n_trial=r.n_trial, margin_chi=r.margin_chi,
               margin_step=r.margin_step, min_pivot=r.min_pivot)
    return res, events


NATIVE_FLAGS = ["-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math"]


def native_lib(dest_dir: Optional[str] = None):
    """The oracle compiled for this host's CPU (gcc -O3 -march=native, still no
    fast-math and no FMA contraction, so every result is the same), for timing
    it as a CPU baseline; built into a temporary directory on first use.
    Returns (library, flags); the portable build if gcc fails."""
    global _native
    if _native is None:
        import tempfile
        d = dest_dir or tempfile.mkdtemp(prefix="oracle_native_")
        path = os.path.join(d, "liboracle_native.so")
        try:
            subprocess.run(["gcc", *NATIVE_FLAGS, "-fPIC", "-shared", "-std=gnu99", "-o", path,
                            SRC_PATH, "-lm", "-lpthread"], check=True, capture_output=True)
            _native = (bind(ctypes.CDLL(path)), " ".join(["gcc", *NATIVE_FLAGS]))
        except (OSError, subprocess.CalledProcessError):
            _native = (lib(), " ".join(["gcc", *PORTABLE_FLAGS]))
    return _native


_native = None


def fit_batch(batch, opts: Optional[Opts] = None, threads: int = 1, library=None) -> dict:
    """Fit every spot of a spotgen.SpotBatch; returns a dict of numpy arrays.
    library: a loaded build of the oracle (default: the portable one)."""
    n = batch.n
    o = opts if opts is not None else default_opts()
    data = np.ascontiguousarray(batch.data)
    if data.dtype == np.uint16:
        dtype = 0
    elif data.dtype == np.float32:
        dtype = 1
    else:
        raise TypeError(data.dtype)
    sizes = np.ascontiguousarray(batch.sizes, dtype=np.uint8)
    offs = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    init = np.ascontiguousarray(batch.init, dtype=np.float32)
    out = dict(params=np.zeros((n, 6)), chi2=np.zeros(n), iters=np.zeros(n, np.int32),
               status=np.zeros(n, np.int32), n_grad=np.zeros(n, np.int32),
               n_trial=np.zeros(n, np.int32), margin_chi=np.zeros(n), margin_step=np.zeros(n),
               min_pivot=np.zeros(n))
    if n == 0:
        return out
    L = library if library is not None else lib()
    rc = L.orc_fit_batch(data.ctypes.data, dtype, sizes.ctypes.data, offs.ctypes.data,
                             init.ctypes.data, n, ctypes.byref(o),
                             *(out[k].ctypes.data for k in ("params", "chi2", "iters", "status",
                                                            "n_grad", "n_trial", "margin_chi",
                                                            "margin_step", "min_pivot")),
                             int(threads))
    if rc != 0:
        raise RuntimeError(f"orc_fit_batch failed ({rc})")
    return out


def moment_init(g, w: int, h: int, model: int) -> np.ndarray:
    """Centroid / second-moment start values of one spot (orc_moment_init)."""
    g = np.ascontiguousarray(g, dtype=np.float64).ravel()
    out = np.empty(4)
    lib().orc_moment_init(_dp(g), int(w), int(h), int(model), _dp(out))
    return out


def moment_init_batch(batch) -> np.ndarray:
    """orc_moment_init over a SpotBatch; float64 [n, 4]."""
    data = np.ascontiguousarray(batch.data)
    dtype = 0 if data.dtype == np.uint16 else 1
    if dtype == 1 and data.dtype != np.float32:
        raise TypeError("data must be uint16 or float32")
    sizes = np.ascontiguousarray(batch.sizes, dtype=np.uint8)
    offs = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    out = np.empty((batch.n, 4))
    lib().orc_moment_init_batch(data.ctypes.data, dtype, sizes.ctypes.data, offs.ctypes.data,
                                int(batch.n), out.ctypes.data)
    return out


def peak_init(g, w: int, h: int) -> np.ndarray:
    """The paper's start values of one spot (orc_peak_init)."""
    g = np.ascontiguousarray(g, dtype=np.float64).ravel()
    out = np.empty(4)
    lib().orc_peak_init(_dp(g), int(w), int(h), _dp(out))
    return out


def peak_init_batch(batch) -> np.ndarray:
    """orc_peak_init over a SpotBatch; float64 [n, 4]."""
    data = np.ascontiguousarray(batch.data)
    dtype = 0 if data.dtype == np.uint16 else 1
    if dtype == 1 and data.dtype != np.float32:
        raise TypeError("data must be uint16 or float32")
    sizes = np.ascontiguousarray(batch.sizes, dtype=np.uint8)
    offs = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    out = np.empty((batch.n, 4))
    lib().orc_peak_init_batch(data.ctypes.data, dtype, sizes.ctypes.data, offs.ctypes.data,
                              int(batch.n), out.ctypes.data)
    return out


def drift_track(params, status, ref_xy, window: int):
    """Drift of fiducial markers over a sequence of frames (the paper's use of the
    fit: tracking markers and averaging their positions over markers and frames to
    stabilise the sample, Introduction).

    params [F, M, 6] and status [F, M]: the fits of M markers in F frames, in
    order; ref_xy [M, 2]: each marker's reference position.  A marker counts in a
    frame when its fit stopped on MAX_ERROR, MIN_DELTA or MIN_STEP with finite x
    and y.  Per frame: (dx, dy) = mean over the counted markers of
    (x - ref_x, y - ref_y) (NaN when none counts); (Dx, Dy) = mean of (dx, dy)
    over those of the last `window` frames (this one included) that had a
    counted marker; n_used, n_frames = the two counts.  Returns float64 [F, 6]
    = (dx, dy, Dx, Dy, n_used, n_frames).
    """
    p = np.asarray(params, dtype=np.float64)
    st = np.asarray(status)
    ref = np.asarray(ref_xy, dtype=np.float64)
    F = p.shape[0]
    out = np.full((F, 6), np.nan)
    per = []
    for f in range(F):
        x, y = p[f, :, 0], p[f, :, 1]
        ok = np.isin(st[f], (MAX_ERROR, MIN_DELTA, MIN_STEP)) & np.isfinite(x) & np.isfinite(y)
        n = int(ok.sum())
        dx = float(np.sum(x[ok] - ref[ok, 0]) / n) if n else np.nan
        dy = float(np.sum(y[ok] - ref[ok, 1]) / n) if n else np.nan
        per.append((dx, dy, n))
        win = [e for e in per[max(0, f - window + 1):] if e[2] > 0]
        out[f, 0], out[f, 1], out[f, 4] = dx, dy, n
        if win:
            out[f, 2] = sum(e[0] for e in win) / len(win)
            out[f, 3] = sum(e[1] for e in win) / len(win)
        out[f, 5] = len(win)
    return out
