"""Host-side checks of the C ABI: the library loads, exports what include/spotfit.h
declares, and rejects bad calls on the host before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_2106_02045_amd as sf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "spotfit.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spotfit_[a-z_0-9]+)\s*\(", text)))


def test_header_declarations_are_exported():
    declared = _declared_functions()
    assert declared, "no declarations found"
    L = sf.lib()
    for name in declared:
        assert hasattr(L, name), f"{name} declared in spotfit.h but not exported"
    assert sorted(sf.EXPORTED) == declared


def test_header_compiles_as_c99(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "spotfit.h"\nint main(void){spotfit_options_t o; (void)o; return 0;}\n')
    import subprocess
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-c",
                        "-I", os.path.join(ROOT, "include"), str(src), "-o",
                        str(tmp_path / "t.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_options_struct_layout_matches_header():
    # offsets of the C struct, checked by compiling a probe against the header
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.c")
        fields = [f for f, _ in sf.Options._fields_]
        body = "".join(f'printf("%zu ", offsetof(spotfit_options_t, {f}));' for f in fields)
        with open(src, "w") as fh:
            fh.write('#include <stdio.h>\n#include <stddef.h>\n#include "spotfit.h"\n'
                     f'int main(void){{{body} printf("%zu", sizeof(spotfit_options_t)); return 0;}}\n')
        exe = os.path.join(d, "p")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    offs = [getattr(sf.Options, f).offset for f in fields]
    assert [int(v) for v in out[:-1]] == offs
    assert int(out[-1]) == ctypes.sizeof(sf.Options)


def test_default_options_are_the_papers():
    o = sf.default_options()
    assert o.max_iter == 20 and o.lambda0_exp10 == -2 and o.lambda_max_exp10 == 4
    assert o.min_delta == 1e-6 and o.min_step_rel == 1e-4
    assert o.max_error_per_px == pytest.approx(1 / 3)
    assert o.max_pixels == 1024 and o.max_side == 32 and o.precision == sf.PREC_FP64
    assert sf.lib().spotfit_validate_options(ctypes.byref(o)) == 0


@pytest.mark.parametrize("field,value", [
    ("max_iter", -1), ("max_iter", 5000), ("precision", 7), ("min_delta", 1.0),
    ("min_delta", -1e-3), ("tie_tau", 1.5), ("sigma_min", 0.0), ("max_pixels", 2000),
    ("max_pixels", 4), ("max_error_per_px", float("nan")), ("sigma_max_frac", 0.05),
    ("max_side", 2), ("max_side", 33), ("schedule", 2), ("plan_hint", 2), ("plan_hint", -1),
])
def test_bad_options_rejected(field, value):
    o = sf.default_options()
    setattr(o, field, value)
    assert sf.lib().spotfit_validate_options(ctypes.byref(o)) == -3
    assert sf.lib().spotfit_last_error()


def test_call_level_errors_before_any_gpu_call():
    L = sf.lib()
    o = sf.default_options()
    # NULL context
    rc = L.spotfit_fit_spots(None, 1, 0, 1, 1, 1, 10, ctypes.byref(o), 1, 1, 1, 1, None, None)
    assert rc == -1
    # a fake non-NULL context is never dereferenced before the argument checks below
    fake = ctypes.c_void_p(0x10)
    assert L.spotfit_fit_spots(fake, 1, 0, 1, 1, 1, -5, ctypes.byref(o), 1, 1, 1, 1, None, None) == -2
    assert L.spotfit_fit_spots(fake, 1, 9, 1, 1, 1, 10, ctypes.byref(o), 1, 1, 1, 1, None, None) == -2
    bad = sf.default_options(max_iter=-3)
    assert L.spotfit_fit_spots(fake, 1, 0, 1, 1, 1, 10, ctypes.byref(bad), 1, 1, 1, 1, None, None) == -3
    # n == 0 is a no-op even with NULL arrays
    assert L.spotfit_fit_spots(fake, None, 0, None, None, None, 0, None, None, None, None, None,
                               None, None) == 0
    # NULL arrays with n > 0
    assert L.spotfit_fit_spots(fake, None, 0, 1, 1, 1, 10, None, 1, 1, 1, 1, None, None) == -1
    assert L.spotfit_fit_spots(fake, 1, 0, 1, 1, 1, 10, None, 1, None, 1, 1, None, None) == -1
    # the raw-spots entry point checks the same way; init_out is required
    args = lambda ctx, n, dt, opt, init_out: (ctx, 1, dt, 1, 1, n, opt, init_out, 1, 1, 1, 1,
                                               None, None)
    assert L.spotfit_fit_raw(*args(None, 10, 0, ctypes.byref(o), 1)) == -1
    assert L.spotfit_fit_raw(*args(fake, -5, 0, ctypes.byref(o), 1)) == -2
    assert L.spotfit_fit_raw(*args(fake, 10, 9, ctypes.byref(o), 1)) == -2
    assert L.spotfit_fit_raw(*args(fake, 10, 0, ctypes.byref(bad), 1)) == -3
    assert L.spotfit_fit_raw(*args(fake, 10, 0, ctypes.byref(o), None)) == -1
    assert L.spotfit_fit_raw(*args(fake, 0, 0, ctypes.byref(o), None)) == 0
    assert L.spotfit_ctx_create(None, 0) == -1
    assert L.spotfit_ctx_reserve(None, 10) == -1
    assert L.spotfit_ctx_reserve(fake, -1) == -2


def test_stats_and_autotune_argument_errors():
    L = sf.lib()
    fake = ctypes.c_void_p(0x10)
    st = sf.Stats()
    assert L.spotfit_get_stats(None, 1, 1, None, 10, ctypes.byref(st), None) == -1
    assert L.spotfit_get_stats(fake, 1, 1, None, 10, None, None) == -1
    assert L.spotfit_get_stats(fake, 1, 1, None, -1, ctypes.byref(st), None) == -2
    assert L.spotfit_get_stats(fake, None, None, None, 0, ctypes.byref(st), None) == 0
    assert st.n_spots == 0 and sum(st.status_count) == 0
    assert L.spotfit_get_stats(fake, None, 1, None, 5, ctypes.byref(st), None) == -1
    o = sf.default_options()
    rep = sf.TuneReport()
    args = (1, 0, 1, 1, 1, 10, ctypes.byref(o), 1, 1, 1, 1)
    assert L.spotfit_autotune(None, *args, 3, ctypes.byref(rep), None) == -1
    assert L.spotfit_autotune(fake, *args, 0, ctypes.byref(rep), None) == -2
    assert L.spotfit_autotune(fake, 1, 0, 1, 1, 1, 0, ctypes.byref(o), 1, 1, 1, 1, 3,
                              ctypes.byref(rep), None) == -2
    p32 = sf.default_options(precision=sf.PREC_FP32)
    assert L.spotfit_autotune(fake, 1, 0, 1, 1, 1, 10, ctypes.byref(p32), 1, 1, 1, 1, 3,
                              ctypes.byref(rep), None) == -3


def test_stats_and_report_struct_layout_matches_header():
    import subprocess
    import tempfile
    checks = [("spotfit_stats_t", sf.Stats), ("spotfit_tune_report_t", sf.TuneReport),
              ("spotfit_frame_t", sf.Frame), ("spotfit_drift_t", sf.Drift),
              ("spotfit_graph_io_t", sf.GraphIO), ("spotfit_serve_stats_t", sf.ServeStats)]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.c")
        body = ""
        for cname, cls in checks:
            for f, _ in cls._fields_:
                body += f'printf("%zu ", offsetof({cname}, {f}));'
            body += f'printf("%zu ", sizeof({cname}));'
        with open(src, "w") as fh:
            fh.write('#include <stdio.h>\n#include <stddef.h>\n#include "spotfit.h"\n'
                     f'int main(void){{{body} return 0;}}\n')
        exe = os.path.join(d, "p")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                              check=True).stdout.split()]
    want = []
    for _, cls in checks:
        want += [getattr(cls, f).offset for f, _ in cls._fields_] + [ctypes.sizeof(cls)]
    assert out == want


def test_version():
    assert sf.version() >= 100


def test_graph_and_tracking_argument_errors():
    # host-side checks only: no HIP call is reached
    L = sf.lib()
    h = ctypes.c_void_p()
    assert L.spotfit_graph_create(None, None, 1, 0, 1, 1, 1, 10, None, 1, 1, 1, 1, None) == -1
    assert L.spotfit_graph_create(ctypes.byref(h), None, 1, 0, 1, 1, 1, 10, None, 1, 1, 1, 1,
                                  None) == -1
    assert h.value is None
    fake = ctypes.c_void_p(0x10)
    # a graph that computes its start values takes no host copy of them
    io = sf.GraphIO(None, 0, 1, None, None, None, None)
    assert L.spotfit_graph_create(ctypes.byref(h), fake, 1, 0, 1, 1, None, 10, None, 1, 1, 1, 1,
                                  ctypes.byref(io)) == -2
    # NULL outputs are still refused when init is NULL
    assert L.spotfit_graph_create(ctypes.byref(h), fake, 1, 0, 1, 1, None, 10, None, None, 1, 1,
                                  1, None) == -1
    assert h.value is None
    assert L.spotfit_graph_launch(None, None) == -1
    L.spotfit_graph_destroy(None)
    assert L.spotfit_serve_track(None, 4, None, 8) == -1


def test_serve_frame_is_validated_before_the_c_call():
    """Server.make_frame checks dtype, shapes and the pixel count the sizes name,
    so the C submit never copies past a host buffer."""
    import numpy as np
    sizes = np.array([[9, 9, 0, 0], [13, 13, 0, 0]], np.uint8)
    npx = 81 + 169
    init = np.zeros((2, 4), np.float32)
    f, _, outs = sf.Server.make_frame(np.zeros(npx, np.uint16), sizes, init)
    assert f.n_spots == 2 and outs["params"].shape == (2, 6)
    sf.Server.make_frame(np.zeros(npx, np.float32), sizes, None)
    for bad in (np.zeros(npx, np.float64), np.zeros(npx, np.int16), np.zeros(npx, np.uint8)):
        with pytest.raises(TypeError):
            sf.Server.make_frame(bad, sizes, init)
    with pytest.raises(ValueError):
        sf.Server.make_frame(np.zeros(npx - 1, np.uint16), sizes, init)
    with pytest.raises(TypeError):
        sf.Server.make_frame(np.zeros(npx, np.uint16), sizes.astype(np.int32), init)
    with pytest.raises(TypeError):
        sf.Server.make_frame(np.zeros(npx, np.uint16), sizes[:, :3], init)
    with pytest.raises(TypeError):
        sf.Server.make_frame(np.zeros(npx, np.uint16), sizes, init[:1])
    with pytest.raises(TypeError):
        sf.Server.make_frame(np.zeros(npx, np.uint16), sizes, init.astype(np.float64))
