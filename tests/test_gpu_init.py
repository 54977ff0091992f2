"""Start values on the device (spotfit_moment_init) against the oracle's estimate,
and the raw-spots-in, fits-out pipeline (needs an MI355X)."""
import numpy as np
import pytest

import oracle
import spotgen
from parity import compare, summary

pytestmark = pytest.mark.gpu


def _up(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda:0"))


def _device_init(ctx, b, **kw):
    import torch

    import paper_2106_02045_amd as sf
    out = ctx.moment_init(_up(b.data), _up(b.sizes), _up(b.offsets), sf.default_options(**kw))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _agree(mine, ref64):
    """float32 results of a double-precision estimate summed in another order:
    equal, or one float32 rounding apart where the double sits on a boundary."""
    ref = ref64.astype(np.float32)
    same = (mine == ref) | (np.isnan(mine) & np.isnan(ref))
    rel = np.abs(mine.astype(np.float64) - ref64) / np.maximum(np.abs(ref64), 1e-30)
    return same.mean(), np.nanmax(np.where(same, 0.0, rel))


@pytest.mark.parametrize("name,side", [("small_11x11", 16), ("mixed_7to32", 32),
                                       ("precision_32x32_ell", 32), ("serve_fiducials", 21)])
def test_device_moment_init_matches_oracle(name, side):
    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload(name, n=8192)
    mine = _device_init(ctx, b, max_side=side)
    ref = oracle.moment_init_batch(b)
    frac, worst = _agree(mine, ref)
    print(f"{name}: {frac:.6f} identical, worst other rel diff {worst:.2e}")
    assert frac >= 0.999 and worst <= 2.0 ** -23


def test_device_moment_init_f32_data_and_unusable_shapes():
    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload("mixed_7to32", n=4096)
    # float data with the background removed (negative values in the ring)
    f = spotgen.SpotBatch(b.data.astype(np.float32) - 300.0, b.sizes.copy(), b.offsets, b.init,
                          b.truth, "f32")
    mine = _device_init(ctx, f, max_side=16)
    ref = oracle.moment_init_batch(f)
    big = np.maximum(f.sizes[:, 0], f.sizes[:, 1]) > 16
    assert np.all(np.isnan(mine[big]))
    frac, worst = _agree(mine[~big], ref[~big])
    assert frac >= 0.999 and worst <= 2.0 ** -23


def test_raw_spots_in_fits_out():
    """Device start values, then the fit: identical decisions to the oracle fit
    started from the same values."""
    import torch

    import paper_2106_02045_amd as sf
    ctx = sf.Context(0)
    b = spotgen.workload("mixed_7to32", n=20000)
    o = sf.default_options(schedule=sf.SCHEDULE_MIXED)
    d = (_up(b.data), _up(b.sizes), _up(b.offsets))
    init = ctx.moment_init(*d, o)
    out = ctx.fit_spots(*d, init, o, want_evals=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    b2 = spotgen.SpotBatch(b.data, b.sizes, b.offsets, init.cpu().numpy(), b.truth, "device init")
    r = oracle.fit_batch(b2, oracle.default_opts(), threads=8)
    c = compare(g, r, chi_band=1e-11, step_band=1e-9)
    print(summary("device init + fit", c))
    assert c["strict_mismatch"] == 0 and c["tol_fail_same"] == 0
