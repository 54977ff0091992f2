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
PREC_FP32, PREC_MIXED, PREC_FP64, PREC_FP32_PLAIN = 0, 1, 2, 3

EXPORTED = ["spotfit_default_options", "spotfit_validate_options", "spotfit_ctx_create",
            "spotfit_ctx_destroy", "spotfit_fit_spots", "spotfit_last_error", "spotfit_version"]


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
    ]


_lib = None


def lib():
    """Load libspotfit.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SpotfitError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
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
        L.spotfit_fit_spots.argtypes = [vp, vp, i32, vp, vp, vp, i64, ctypes.POINTER(Options),
                                        vp, vp, vp, vp, vp, vp]
        L.spotfit_fit_spots.restype = ctypes.c_int
        L.spotfit_last_error.argtypes = []
        L.spotfit_last_error.restype = ctypes.c_char_p
        L.spotfit_version.argtypes = []
        L.spotfit_version.restype = ctypes.c_int
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

    def fit_spots(self, data, sizes, offsets, init, opts: Optional[Options] = None,
                  out=None, want_evals: bool = False, stream=None):
        """Fit spots held in torch CUDA tensors; returns a dict of output tensors.

        data: uint16 or float32 [total pixels]; sizes: uint8 [n, 4]; offsets: int64 [n];
        init: float32 [n, 4].  Outputs are allocated with torch unless `out` supplies
        them (dict with params, chi2, iters, status[, evals]).  Enqueued on `stream`
        (default: torch's current stream); synchronise before reading the outputs.
        """
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
            if t.dtype != want or not t.is_contiguous() or t.device != dev:
                raise TypeError(f"{name} must be a contiguous {want} tensor on {dev}")
        if not data.is_contiguous():
            raise TypeError("data must be contiguous")
        if sizes.dim() != 2 or sizes.shape[1] != 4 or init.shape != (n, 4) or offsets.shape != (n,):
            raise ValueError("shape mismatch: sizes [n,4], offsets [n], init [n,4]")
        if out is None:
            out = dict(params=torch.empty((n, 6), dtype=torch.float32, device=dev),
                       chi2=torch.empty(n, dtype=torch.float32, device=dev),
                       iters=torch.empty(n, dtype=torch.int32, device=dev),
                       status=torch.empty(n, dtype=torch.int32, device=dev))
            if want_evals:
                out["evals"] = torch.empty((n, 2), dtype=torch.int32, device=dev)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        rc = self.fit_spots_raw(data.data_ptr(), dt, sizes.data_ptr(), offsets.data_ptr(),
                                init.data_ptr(), n, opts, out["params"].data_ptr(),
                                out["chi2"].data_ptr(), out["iters"].data_ptr(),
                                out["status"].data_ptr(),
                                out["evals"].data_ptr() if "evals" in out else 0,
                                st.cuda_stream)
        _check(rc, "spotfit_fit_spots")
        return out


def version() -> int:
    return int(lib().spotfit_version())
