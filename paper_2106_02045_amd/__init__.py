"""MI355X-native batched Gaussian-spot fitting (implicit-amplitude Levenberg-Marquardt).

Thin ctypes binding of the C ABI in include/spotfit.h.  It only marshals
arguments: every step of the fit runs in the HIP kernels of libspotfit.so.
If the library is missing the binding raises; there is no CPU fallback.
PyTorch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspotfit.so")

U16, F32 = 0, 1
SYM, ELL = 0, 1
MAX_ITER, MAX_ERROR, MIN_DELTA, MIN_STEP, NOT_CONVERGED, BAD_INPUT = range(6)
STATUS_NAMES = ["MAX_ITER", "MAX_ERROR", "MIN_DELTA", "MIN_STEP", "NOT_CONVERGED", "BAD_INPUT"]
PREC_FP32, PREC_MIXED, PREC_FP64, PREC_FP32_PLAIN, PREC_COMP = 0, 1, 2, 3, 4
SCHEDULE_UNIFORM, SCHEDULE_MIXED = 0, 1
PLAN_THROUGHPUT, PLAN_LATENCY = 0, 1

EXPORTED = ["spotfit_default_options", "spotfit_validate_options", "spotfit_ctx_create",
            "spotfit_ctx_destroy", "spotfit_ctx_reserve", "spotfit_fit_spots",
            "spotfit_last_error", "spotfit_version", "spotfit_serve_create",
            "spotfit_serve_submit", "spotfit_serve_poll", "spotfit_serve_wait",
            "spotfit_serve_stats", "spotfit_serve_destroy", "spotfit_serve_replay",
            "spotfit_serve_last_error", "spotfit_get_stats", "spotfit_autotune",
            "spotfit_moment_init", "spotfit_peak_init", "spotfit_serve_track",
            "spotfit_graph_create", "spotfit_graph_launch", "spotfit_graph_destroy",
            "spotfit_fit_raw", "spotfit_fit_spots_noalloc", "spotfit_exp_neg"]
E_AGAIN = -6
NOALLOC_MAX_SPOTS = 1 << 20


class SpotfitError(RuntimeError):
    pass


class Options(ctypes.Structure):
    """Mirror of spotfit_options_t."""
    _fields_ = [
        ("max_iter", ctypes.c_int32),
        ("lambda0_exp10", ctypes.c_int32),
        ("lambda_max_exp10", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_error_per_px", ctypes.c_double),
        ("min_delta", ctypes.c_double),
        ("min_step_rel", ctypes.c_double),
        ("tie_tau", ctypes.c_double),
        ("sigma_min", ctypes.c_double),
        ("sigma_max_frac", ctypes.c_double),
        ("max_pixels", ctypes.c_int32),
        ("max_side", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("plan_hint", ctypes.c_int32),
    ]


class GraphIO(ctypes.Structure):
    """Mirror of spotfit_graph_io_t (pinned host pointers or NULL)."""
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("data_bytes", ctypes.c_int64),
        ("init", ctypes.c_void_p),
        ("params", ctypes.c_void_p),
        ("chi2", ctypes.c_void_p),
        ("iters", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


class Drift(ctypes.Structure):
    """Mirror of spotfit_drift_t."""
    _fields_ = [
        ("dx", ctypes.c_float),
        ("dy", ctypes.c_float),
        ("mean_dx", ctypes.c_float),
        ("mean_dy", ctypes.c_float),
        ("n_used", ctypes.c_int32),
        ("n_frames", ctypes.c_int32),
    ]


DRIFT_DTYPE = [("dx", "<f4"), ("dy", "<f4"), ("mean_dx", "<f4"), ("mean_dy", "<f4"),
               ("n_used", "<i4"), ("n_frames", "<i4")]


class Frame(ctypes.Structure):
    """Mirror of spotfit_frame_t (host pointers)."""
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("sizes", ctypes.c_void_p),
        ("init", ctypes.c_void_p),
        ("n_spots", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("params_out", ctypes.c_void_p),
        ("chi2_out", ctypes.c_void_p),
        ("iters_out", ctypes.c_void_p),
        ("status_out", ctypes.c_void_p),
        ("drift_out", ctypes.c_void_p),
    ]


class ServeStats(ctypes.Structure):
    """Mirror of spotfit_serve_stats_t."""
    _fields_ = [
        ("frames_done", ctypes.c_uint64),
        ("frames_failed", ctypes.c_uint64),
        ("spots_done", ctypes.c_uint64),
        ("batches", ctypes.c_uint64),
        ("rejected", ctypes.c_uint64),
        ("latency_p50_us", ctypes.c_double),
        ("latency_p99_us", ctypes.c_double),
        ("latency_max_us", ctypes.c_double),
        ("mean_frames_per_batch", ctypes.c_double),
        ("wall_s", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    """Mirror of spotfit_stats_t."""
    _fields_ = [
        ("n_spots", ctypes.c_int64),
        ("status_count", ctypes.c_int64 * 6),
        ("iters_hist", ctypes.c_int64 * 65),
        ("grad_evals", ctypes.c_int64),
        ("trial_evals", ctypes.c_int64),
    ]


class TuneReport(ctypes.Structure):
    """Mirror of spotfit_tune_report_t."""
    _fields_ = [
        ("schedule", ctypes.c_int32),
        ("size_class", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32),
        ("chosen", ctypes.c_int32),
        ("plan_id", ctypes.c_int32 * 16),
        ("plan_ms", ctypes.c_double * 16),
    ]


_lib = None


def lib():
    """Load libspotfit.so (built by paper_2106_02045_amd/build.py); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SpotfitError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_2106_02045_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.spotfit_default_options.argtypes = [ctypes.POINTER(Options)]
        L.spotfit_default_options.restype = None
        L.spotfit_validate_options.argtypes = [ctypes.POINTER(Options)]
        L.spotfit_validate_options.restype = ctypes.c_int
        L.spotfit_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.spotfit_ctx_create.restype = ctypes.c_int
        L.spotfit_ctx_destroy.argtypes = [vp]
        L.spotfit_ctx_destroy.restype = None
        L.spotfit_ctx_reserve.argtypes = [vp, i64]
        L.spotfit_ctx_reserve.restype = ctypes.c_int
        L.spotfit_fit_spots.argtypes = [vp, vp, i32, vp, vp, vp, i64, ctypes.POINTER(Options),
                                        vp, vp, vp, vp, vp, vp]
        L.spotfit_fit_spots.restype = ctypes.c_int
        L.spotfit_fit_spots_noalloc.argtypes = L.spotfit_fit_spots.argtypes
        L.spotfit_fit_spots_noalloc.restype = ctypes.c_int
        L.spotfit_exp_neg.argtypes = [vp, vp, i64, vp]
        L.spotfit_exp_neg.restype = ctypes.c_int
        L.spotfit_fit_raw.argtypes = [vp, vp, i32, vp, vp, i64, ctypes.POINTER(Options), vp,
                                      vp, vp, vp, vp, vp, vp]
        L.spotfit_fit_raw.restype = ctypes.c_int
        L.spotfit_last_error.argtypes = []
        L.spotfit_last_error.restype = ctypes.c_char_p
        L.spotfit_version.argtypes = []
        L.spotfit_version.restype = ctypes.c_int
        u64 = ctypes.c_uint64
        L.spotfit_serve_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int,
                                           ctypes.POINTER(Options), ctypes.c_size_t, i32, i32]
        L.spotfit_serve_create.restype = ctypes.c_int
        L.spotfit_serve_submit.argtypes = [vp, ctypes.POINTER(Frame), u64, ctypes.POINTER(u64)]
        L.spotfit_serve_submit.restype = ctypes.c_int
        L.spotfit_serve_poll.argtypes = [vp, u64]
        L.spotfit_serve_poll.restype = ctypes.c_int
        L.spotfit_serve_wait.argtypes = [vp, u64]
        L.spotfit_serve_wait.restype = ctypes.c_int
        L.spotfit_serve_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
        L.spotfit_serve_track.argtypes = [vp, i32, vp, i32]
        L.spotfit_serve_track.restype = ctypes.c_int
        L.spotfit_graph_create.argtypes = [ctypes.POINTER(vp), vp, vp, i32, vp, vp, vp, i64,
                                           ctypes.POINTER(Options), vp, vp, vp, vp,
                                           ctypes.POINTER(GraphIO)]
        L.spotfit_graph_create.restype = ctypes.c_int
        L.spotfit_graph_launch.argtypes = [vp, vp]
        L.spotfit_graph_launch.restype = ctypes.c_int
        L.spotfit_graph_destroy.argtypes = [vp]
        L.spotfit_graph_destroy.restype = None
        L.spotfit_serve_stats.restype = ctypes.c_int
        L.spotfit_serve_destroy.argtypes = [vp]
        L.spotfit_serve_destroy.restype = None
        L.spotfit_serve_replay.argtypes = [vp, ctypes.POINTER(Frame), i64, vp]
        L.spotfit_serve_replay.restype = ctypes.c_int
        L.spotfit_serve_last_error.argtypes = []
        L.spotfit_serve_last_error.restype = ctypes.c_char_p
        L.spotfit_moment_init.argtypes = [vp, vp, i32, vp, vp, i64, ctypes.POINTER(Options), vp,
                                          vp]
        L.spotfit_moment_init.restype = ctypes.c_int
        L.spotfit_peak_init.argtypes = L.spotfit_moment_init.argtypes
        L.spotfit_peak_init.restype = ctypes.c_int
        L.spotfit_get_stats.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(Stats), vp]
        L.spotfit_get_stats.restype = ctypes.c_int
        L.spotfit_autotune.argtypes = [vp, vp, i32, vp, vp, vp, i64, ctypes.POINTER(Options),
                                       vp, vp, vp, vp, i32, ctypes.POINTER(TuneReport), vp]
        L.spotfit_autotune.restype = ctypes.c_int
        _lib = L
    return _lib


def default_options(**kw) -> Options:
    o = Options()
    lib().spotfit_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().spotfit_last_error().decode(errors="replace")
        raise SpotfitError(f"{what} failed with {rc}: {msg}")


class Context:
    """A spotfit_ctx_t on one device (kernel plans, device properties)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().spotfit_ctx_create(ctypes.byref(h), int(device)), "spotfit_ctx_create")
        self._h = h
        self.device = int(device)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().spotfit_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, n_spots: int):
        """Size the device workspace for mixed-schedule calls of up to n_spots spots."""
        _check(lib().spotfit_ctx_reserve(self._h, int(n_spots)), "spotfit_ctx_reserve")

    def fit_spots_raw(self, data_ptr: int, dtype: int, sizes_ptr: int, offsets_ptr: int,
                      init_ptr: int, n: int, opts: Optional[Options], params_ptr: int,
                      chi2_ptr: int, iters_ptr: int, status_ptr: int, evals_ptr: int,
                      stream_ptr: int) -> int:
        """Direct C-ABI call with raw device pointers; returns the C return code."""
        return lib().spotfit_fit_spots(self._h, data_ptr, dtype, sizes_ptr, offsets_ptr,
                                       init_ptr, int(n),
                                       ctypes.byref(opts) if opts is not None else None,
                                       params_ptr, chi2_ptr, iters_ptr, status_ptr,
                                       evals_ptr or None, stream_ptr or None)

    @staticmethod
    def _marshal(data, sizes, offsets, init, out, want_evals):
        import torch
        n = int(sizes.shape[0])
        dev = data.device
        if data.dtype == torch.uint16:
            dt = U16
        elif data.dtype == torch.float32:
            dt = F32
        else:
            raise TypeError(f"data must be uint16 or float32, got {data.dtype}")
        for name, t, want in (("sizes", sizes, torch.uint8), ("offsets", offsets, torch.int64),
                              ("init", init, torch.float32)):
            if t is None and name == "init":
                continue
            if t.dtype != want or not t.is_contiguous() or t.device != dev:
                raise TypeError(f"{name} must be a contiguous {want} tensor on {dev}")
        if not data.is_contiguous():
            raise TypeError("data must be contiguous")
        if (sizes.dim() != 2 or sizes.shape[1] != 4 or offsets.shape != (n,)
                or (init is not None and init.shape != (n, 4))):
            raise ValueError("shape mismatch: sizes [n,4], offsets [n], init [n,4]")
        if out is None:
            out = dict(params=torch.empty((n, 6), dtype=torch.float32, device=dev),
                       chi2=torch.empty(n, dtype=torch.float32, device=dev),
                       iters=torch.empty(n, dtype=torch.int32, device=dev),
                       status=torch.empty(n, dtype=torch.int32, device=dev))
            if want_evals:
                out["evals"] = torch.empty((n, 2), dtype=torch.int32, device=dev)
        else:
            want = dict(params=((n, 6), torch.float32), chi2=((n,), torch.float32),
                        iters=((n,), torch.int32), status=((n,), torch.int32),
                        evals=((n, 2), torch.int32))
            for k, (shape, dtype) in want.items():
                if k not in out:
                    if k == "evals":
                        continue
                    raise ValueError(f"out is missing {k}")
                t = out[k]
                if (tuple(t.shape) != shape or t.dtype != dtype or not t.is_contiguous()
                        or t.device != dev):
                    raise TypeError(f"out[{k!r}] must be a contiguous {dtype} tensor of shape "
                                    f"{shape} on {dev}")
        return n, dt, out

    def fit_spots(self, data, sizes, offsets, init, opts: Optional[Options] = None,
                  out=None, want_evals: bool = False, stream=None):
        """Fit spots held in torch CUDA tensors; returns a dict of output tensors.

        data: uint16 or float32 [total pixels]; sizes: uint8 [n, 4]; offsets: int64 [n];
        init: float32 [n, 4].  Outputs are allocated with torch unless `out` supplies
        them (dict with params, chi2, iters, status[, evals]).  Enqueued on `stream`
        (default: torch's current stream); synchronise before reading the outputs.
        """
        import torch
        n, dt, out = self._marshal(data, sizes, offsets, init, out, want_evals)
        st = stream if stream is not None else torch.cuda.current_stream(data.device)
        rc = self.fit_spots_raw(data.data_ptr(), dt, sizes.data_ptr(), offsets.data_ptr(),
                                init.data_ptr(), n, opts, out["params"].data_ptr(),
                                out["chi2"].data_ptr(), out["iters"].data_ptr(),
                                out["status"].data_ptr(),
                                out["evals"].data_ptr() if "evals" in out else 0,
                                st.cuda_stream)
        _check(rc, "spotfit_fit_spots")
        return out

    def fit_spots_noalloc(self, data, sizes, offsets, init, opts: Optional[Options] = None,
                          out=None, want_evals: bool = False, stream=None):
        """spotfit_fit_spots_noalloc: fit_spots whose counters and size-class lists are
        the library's fixed device array instead of the context's workspace.  `out`
        should be supplied by callers that must not allocate (otherwise torch
        allocates the outputs here)."""
        import torch
        n, dt, out = self._marshal(data, sizes, offsets, init, out, want_evals)
        st = stream if stream is not None else torch.cuda.current_stream(data.device)
        rc = lib().spotfit_fit_spots_noalloc(
            self._h, data.data_ptr(), dt, sizes.data_ptr(), offsets.data_ptr(),
            init.data_ptr(), n, ctypes.byref(opts) if opts is not None else None,
            out["params"].data_ptr(), out["chi2"].data_ptr(), out["iters"].data_ptr(),
            out["status"].data_ptr(), (out["evals"].data_ptr() if "evals" in out else 0) or None,
            st.cuda_stream or None)
        _check(rc, "spotfit_fit_spots_noalloc")
        return out

    def fit_raw(self, data, sizes, offsets, opts: Optional[Options] = None, out=None,
                want_evals: bool = False, stream=None):
        """Raw spots in, fits out (spotfit_fit_raw): the centroid / second-moment start
        values and the fit from them, in the fit's own launch with the double-precision
        kernels.  Returns fit_spots' outputs plus "init", float32 [n, 4]: the start
        values each fit began from.  `out` may supply any of the outputs, "init" too."""
        import torch
        n = int(sizes.shape[0])
        out = dict(out) if out is not None else {}
        init = out.pop("init", None)
        if init is None:
            init = torch.empty((n, 4), dtype=torch.float32, device=data.device)
        n, dt, res = self._marshal(data, sizes, offsets, init, out or None, want_evals)
        st = stream if stream is not None else torch.cuda.current_stream(data.device)
        rc = lib().spotfit_fit_raw(self._h, data.data_ptr(), dt, sizes.data_ptr(),
                                   offsets.data_ptr(), n,
                                   ctypes.byref(opts) if opts is not None else None,
                                   init.data_ptr(), res["params"].data_ptr(),
                                   res["chi2"].data_ptr(), res["iters"].data_ptr(),
                                   res["status"].data_ptr(),
                                   res["evals"].data_ptr() if "evals" in res else None,
                                   st.cuda_stream or None)
        _check(rc, "spotfit_fit_raw")
        res["init"] = init
        return res

    def graph(self, data, sizes, offsets, init, opts: Optional[Options] = None, out=None,
              host=None):
        """Capture one fit of this fixed batch into a HIP graph (spotfit_graph_create).

        The device tensors (and `out`, allocated if None) are baked into the graph: refill
        them between launches.  host: optional dict of PINNED CPU tensors with keys
        data, init (copied to the device before the fit) and params, chi2, iters, status
        (copied back after it).  init None: the graph computes the start values on the
        device (as fit_raw does) and a replay takes raw pixels to fits.  Returns a Graph
        whose launch() replays the whole call."""
        n, dt, out = self._marshal(data, sizes, offsets, init, out, False)
        if init is None and host and "init" in host:
            raise ValueError("host['init'] needs a device init tensor")
        io = None
        host = dict(host or {})
        if host:
            for k, t in host.items():
                if k not in ("data", "init", "params", "chi2", "iters", "status"):
                    raise KeyError(k)
                if t.is_cuda or not t.is_pinned() or not t.is_contiguous():
                    raise TypeError(f"host[{k!r}] must be a contiguous pinned CPU tensor")
            for k in ("init", "params", "chi2", "iters", "status"):
                ref = init if k == "init" else out[k]
                if k in host and ref is not None and (host[k].shape != ref.shape
                                                      or host[k].dtype != ref.dtype):
                    raise ValueError(f"host[{k!r}] must match {tuple(ref.shape)} {ref.dtype}")
            if "data" in host and (host["data"].dtype != data.dtype
                                   or host["data"].numel() != data.numel()):
                raise ValueError("host['data'] must match the device data")
            ptr = lambda k: host[k].data_ptr() if k in host else None
            io = GraphIO(ptr("data"), host["data"].numel() * host["data"].element_size()
                         if "data" in host else 0, ptr("init"), ptr("params"), ptr("chi2"),
                         ptr("iters"), ptr("status"))
        h = ctypes.c_void_p()
        rc = lib().spotfit_graph_create(ctypes.byref(h), self._h, data.data_ptr(), dt,
                                        sizes.data_ptr(), offsets.data_ptr(),
                                        init.data_ptr() if init is not None else None, n,
                                        ctypes.byref(opts) if opts is not None else None,
                                        out["params"].data_ptr(), out["chi2"].data_ptr(),
                                        out["iters"].data_ptr(), out["status"].data_ptr(),
                                        ctypes.byref(io) if io is not None else None)
        _check(rc, "spotfit_graph_create")
        return Graph(h, keep=(data, sizes, offsets, init, out, host, io), out=out)

    def autotune(self, data, sizes, offsets, init, opts: Optional[Options] = None, reps: int = 3,
                 out=None, stream=None):
        """Time every lane mapping on this batch and keep the fastest (spotfit_autotune).

        Returns (outputs of the kept plan, report dict with plan ids, ms per call, chosen)."""
        import torch
        n, dt, out = self._marshal(data, sizes, offsets, init, out, False)
        st = stream if stream is not None else torch.cuda.current_stream(data.device)
        rep = TuneReport()
        rc = lib().spotfit_autotune(self._h, data.data_ptr(), dt, sizes.data_ptr(),
                                    offsets.data_ptr(), init.data_ptr(), n,
                                    ctypes.byref(opts) if opts is not None else None,
                                    out["params"].data_ptr(), out["chi2"].data_ptr(),
                                    out["iters"].data_ptr(), out["status"].data_ptr(), int(reps),
                                    ctypes.byref(rep), st.cuda_stream)
        _check(rc, "spotfit_autotune")
        k = rep.n_candidates
        report = dict(schedule=rep.schedule, size_class=rep.size_class,
                      plan_id=list(rep.plan_id[:k]), plan_ms=list(rep.plan_ms[:k]),
                      chosen_plan=rep.plan_id[rep.chosen])
        return out, report

    def _start_values(self, fn: str, data, sizes, offsets, opts, out, stream):
        import torch
        n = int(sizes.shape[0])
        dt = U16 if data.dtype == torch.uint16 else F32 if data.dtype == torch.float32 else None
        if dt is None:
            raise TypeError(f"data must be uint16 or float32, got {data.dtype}")
        for name, t, want in (("sizes", sizes, torch.uint8), ("offsets", offsets, torch.int64)):
            if t.dtype != want or not t.is_contiguous() or t.device != data.device:
                raise TypeError(f"{name} must be a contiguous {want} tensor on {data.device}")
        if tuple(sizes.shape) != (n, 4) or tuple(offsets.shape) != (n,):
            raise ValueError("sizes must be [n, 4] and offsets [n]")
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=data.device)
        elif (out.dtype != torch.float32 or tuple(out.shape) != (n, 4) or not out.is_contiguous()
              or out.device != data.device):
            raise TypeError(f"out must be a contiguous float32 [n, 4] tensor on {data.device}")
        st = stream if stream is not None else torch.cuda.current_stream(data.device)
        rc = getattr(lib(), fn)(self._h, data.data_ptr(), dt, sizes.data_ptr(),
                                offsets.data_ptr(), n,
                                ctypes.byref(opts) if opts is not None else None,
                                out.data_ptr(), st.cuda_stream)
        _check(rc, fn)
        return out

    def moment_init(self, data, sizes, offsets, opts: Optional[Options] = None, out=None,
                    stream=None):
        """Centroid / second-moment start values on the device (spotfit_moment_init);
        returns float32 [n, 4]."""
        return self._start_values("spotfit_moment_init", data, sizes, offsets, opts, out, stream)

    def peak_init(self, data, sizes, offsets, opts: Optional[Options] = None, out=None,
                  stream=None):
        """The paper's start values on the device (spotfit_peak_init): brightest pixel of
        the 3x3 moving average, sigma = sqrt(M / pi); returns float32 [n, 4]."""
        return self._start_values("spotfit_peak_init", data, sizes, offsets, opts, out, stream)

    def stats(self, out, stream=None):
        """Stop reasons, iteration histogram and evaluation totals of a fit's outputs."""
        import torch
        n = int(out["status"].shape[0])
        st = stream if stream is not None else torch.cuda.current_stream(out["status"].device)
        res = Stats()
        rc = lib().spotfit_get_stats(self._h, out["status"].data_ptr(), out["iters"].data_ptr(),
                                     out["evals"].data_ptr() if "evals" in out else None, n,
                                     ctypes.byref(res), st.cuda_stream)
        _check(rc, "spotfit_get_stats")
        return dict(n_spots=res.n_spots, status_count=list(res.status_count),
                    iters_hist=list(res.iters_hist), grad_evals=res.grad_evals,
                    trial_evals=res.trial_evals)


class Graph:
    """A captured fit (spotfit_graph_t); holds the tensors baked into it."""

    def __init__(self, h, keep, out):
        self._h = h
        self._keep = keep
        self.out = out

    def launch(self, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self.out["params"].device)
        _check(lib().spotfit_graph_launch(self._h, st.cuda_stream), "spotfit_graph_launch")

    def close(self):
        if self._h:
            lib().spotfit_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exp_neg(x, stream=None):
    """e^x (x <= 0) by the fit kernels' own exponential (spotfit_exp_neg), for a
    float64 torch CUDA tensor; returns a new tensor."""
    import torch
    if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a contiguous float64 CUDA tensor")
    y = torch.empty_like(x)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    _check(lib().spotfit_exp_neg(x.data_ptr(), y.data_ptr(), x.numel(), st.cuda_stream or None),
           "spotfit_exp_neg")
    return y


def version() -> int:
    return int(lib().spotfit_version())


class Server:
    """Real-time serving loop (spotfit_serve_t): frames from host memory in, fits out.

    Frames are numpy arrays on the host; results land in numpy arrays that this
    object keeps alive until the frame is done.
    """

    def __init__(self, device: int = 0, opts: Optional[Options] = None,
                 device_mem_budget: int = 256 << 20, max_frames: int = 4096, n_streams: int = 2):
        h = ctypes.c_void_p()
        rc = lib().spotfit_serve_create(ctypes.byref(h), int(device),
                                        ctypes.byref(opts) if opts is not None else None,
                                        int(device_mem_budget), int(max_frames), int(n_streams))
        if rc != 0:
            raise SpotfitError(f"spotfit_serve_create failed with {rc}: "
                               f"{lib().spotfit_serve_last_error().decode(errors='replace')}")
        self._h = h
        self._keep = {}

    def track(self, ref_xy, window: int):
        """Turn on drift tracking (spotfit_serve_track): ref_xy [M, 2] reference marker
        positions; frames submitted with track=True then carry outputs["drift"].
        ref_xy None turns it off.  Call with no frame in flight."""
        import numpy as np
        if ref_xy is None:
            m, ptr = 0, None
        else:
            ref = np.ascontiguousarray(ref_xy, dtype=np.float32)
            if ref.ndim != 2 or ref.shape[1] != 2:
                raise ValueError("ref_xy must be [n_markers, 2]")
            m, ptr = int(ref.shape[0]), ref.ctypes.data
        rc = lib().spotfit_serve_track(self._h, m, ptr, int(window))
        if rc != 0:
            raise SpotfitError(f"spotfit_serve_track failed with {rc}: "
                               f"{lib().spotfit_serve_last_error().decode(errors='replace')}")

    @staticmethod
    def make_frame(data, sizes, init, track: bool = False):
        """Build a spotfit_frame_t (and its output arrays) from numpy arrays.
        init None: start values computed on the device.  track: a tracked frame,
        whose drift record lands in outputs["drift"] (a structured array of one)."""
        import numpy as np
        data = np.ascontiguousarray(data)
        if data.dtype not in (np.uint16, np.float32):
            raise TypeError(f"frame data must be uint16 or float32, got {data.dtype}")
        sizes = np.asarray(sizes)
        if sizes.dtype != np.uint8 or sizes.ndim != 2 or sizes.shape[1] != 4:
            raise TypeError("frame sizes must be a uint8 array of shape [n, 4]")
        sizes = np.ascontiguousarray(sizes)
        n = int(sizes.shape[0])
        npx = int((sizes[:, 0].astype(np.int64) * sizes[:, 1].astype(np.int64)).sum())
        if data.ndim != 1 or data.size < npx:
            raise ValueError(f"frame data must be flat and hold the {npx} pixels its sizes name, "
                             f"got shape {data.shape}")
        if init is not None:
            init = np.asarray(init)
            if init.dtype != np.float32 or init.shape != (n, 4):
                raise TypeError(f"frame init must be float32 of shape ({n}, 4)")
            init = np.ascontiguousarray(init)
        outs = dict(params=np.zeros((n, 6), np.float32), chi2=np.zeros(n, np.float32),
                    iters=np.zeros(n, np.int32), status=np.zeros(n, np.int32))
        if track:
            outs["drift"] = np.zeros(1, dtype=DRIFT_DTYPE)
        f = Frame(data.ctypes.data, sizes.ctypes.data,
                  init.ctypes.data if init is not None else None, n,
                  U16 if data.dtype == np.uint16 else F32, outs["params"].ctypes.data,
                  outs["chi2"].ctypes.data, outs["iters"].ctypes.data, outs["status"].ctypes.data,
                  outs["drift"].ctypes.data if track else None)
        return f, (data, sizes, init), outs

    def submit(self, data, sizes, init, arrival_ns: int = 0, track: bool = False):
        """Returns (ticket, outputs) or None when the frame is not admitted now."""
        f, ins, outs = self.make_frame(data, sizes, init, track)
        t = ctypes.c_uint64()
        rc = lib().spotfit_serve_submit(self._h, ctypes.byref(f), int(arrival_ns), ctypes.byref(t))
        if rc == E_AGAIN:
            return None
        if rc != 0:
            raise SpotfitError(f"spotfit_serve_submit failed with {rc}: "
                               f"{lib().spotfit_serve_last_error().decode(errors='replace')}")
        self._keep[t.value] = outs
        return t.value, outs

    def wait(self, ticket: int):
        """Block until the frame is done; its outputs, or SpotfitError if it failed."""
        rc = lib().spotfit_serve_wait(self._h, int(ticket))
        if rc != 0:
            self._keep.pop(ticket, None)
            raise SpotfitError(f"spotfit_serve_wait failed with {rc}: "
                               f"{lib().spotfit_serve_last_error().decode(errors='replace')}")
        return self._keep.pop(ticket)

    def poll(self, ticket: int) -> int:
        return lib().spotfit_serve_poll(self._h, int(ticket))

    def replay(self, frames, arrival_offset_ns):
        """frames: list of (data, sizes, init[, track]); arrival offsets in ns.  Returns
        outputs."""
        import numpy as np
        built = [self.make_frame(*fr) for fr in frames]
        arr = (Frame * len(built))(*[b[0] for b in built])
        offs = np.ascontiguousarray(arrival_offset_ns, dtype=np.uint64)
        rc = lib().spotfit_serve_replay(self._h, arr, len(built), offs.ctypes.data)
        if rc != 0:
            raise SpotfitError(f"spotfit_serve_replay failed with {rc}: "
                               f"{lib().spotfit_serve_last_error().decode(errors='replace')}")
        return [b[2] for b in built]

    def stats(self) -> dict:
        st = ServeStats()
        _check(lib().spotfit_serve_stats(self._h, ctypes.byref(st)), "spotfit_serve_stats")
        return {k: getattr(st, k) for k, _ in ServeStats._fields_}

    def close(self):
        if self._h:
            lib().spotfit_serve_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
