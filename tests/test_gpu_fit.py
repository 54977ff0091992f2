"""GPU fit vs the double-precision oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import spotgen
from parity import compare, summary

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    dev = torch.device("cuda:0")

    def run(batch, **kw):
        up = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        o = sf.default_options(**kw)
        out = ctx.fit_spots(up(batch.data), up(batch.sizes), up(batch.offsets), up(batch.init), o,
                            want_evals=True)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    return run


TAU = 9e-7


def test_small_workload_mixed_precision(gpu):
    b = spotgen.config(0)
    g = gpu(b, tie_tau=TAU, max_pixels=121)
    r = oracle.fit_batch(b, oracle.default_opts(tie_tau=TAU), threads=8)
    c = compare(g, r, chi_band=3e-6, step_band=1e-2)
    print(summary("small 11x11 mixed", c))
    assert c["tol_fail_same"] == 0
    assert c["status_mismatch"] <= 0.05 * b.n
    np.testing.assert_array_equal(g["evals"][:, 0][g["status"] == r["status"]],
                                  r["n_grad"][g["status"] == r["status"]])


def test_small_workload_fp32(gpu):
    b = spotgen.config(0)
    g = gpu(b, tie_tau=TAU, max_pixels=121, precision=0)
    r = oracle.fit_batch(b, oracle.default_opts(tie_tau=TAU), threads=8)
    c = compare(g, r, chi_band=3e-6, step_band=1e-2)
    print(summary("small 11x11 fp32", c))
    assert c["max_dxy"] < 1e-3
    assert c["status_mismatch"] <= 0.1 * b.n


def test_run_to_run_bitwise(gpu):
    b = spotgen.config(3, n=3000)
    g1 = gpu(b)
    g2 = gpu(b)
    for k in g1:
        np.testing.assert_array_equal(g1[k], g2[k])


def test_bad_inputs_flagged(gpu):
    b = spotgen.config(0, n=8)
    b.sizes[1, 2] = 7          # unknown model
    b.init[2, 2] = 0.0         # sigma <= 0
    b.init[3, 0] = np.nan      # non-finite start
    b.sizes[4, 0] = 2          # w < 3 (pixels of the spot stay where they are)
    g = gpu(b, max_pixels=121)
    for s in (1, 2, 3, 4):
        assert g["status"][s] == 5 and g["iters"][s] == 0
        assert np.all(np.isnan(g["params"][s]))
    assert np.all(g["status"][[0, 5, 6, 7]] != 5)


def test_capacity_promise(gpu):
    b = spotgen.config(3, n=400)
    g = gpu(b, max_pixels=121)
    big = b.npix() > 121
    assert np.all(g["status"][big] == 5)
    assert np.all(g["status"][~big] != 5)
