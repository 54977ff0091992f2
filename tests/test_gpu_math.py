"""The fit kernels' own exponential (spotfit_exp_neg: Cody-Waite reduction, Taylor
series of degree 13, scaling by 2^n) against the C library's exp, over the range
the profile factors of Eq. 10 take (x <= 0), through the C ABI (needs an MI355X).

The reference is the exponential in x87 extended precision (64-bit significand,
numpy longdouble), rounded to double: the correctly rounded value except within
~2^-11 ulp of a rounding boundary.  The bound: the device value's error against
the extended value is below 1 ulp wherever the result is normal, so it is the
correctly rounded double or a neighbour (the reduction's residual and the
truncated series each contribute well under an ulp); exactly 1 at 0, monotone
non-increasing on a fine grid, and 0 or subnormal below the double range, with
NaN kept.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _dev_exp(x):
    import torch

    import paper_2106_02045_amd as sf
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(torch.device("cuda:0"))
    y = sf.exp_neg(t)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _ulps(a, b):
    """|a - b| in units of the spacing of doubles at b."""
    return np.abs(a - b) / np.spacing(np.abs(b))


def test_exp_neg_within_one_ulp():
    rng = np.random.default_rng(2106)
    x = np.concatenate([
        -rng.uniform(0.0, 1.0, 400000),            # near the peak of the profile
        -rng.uniform(0.0, 50.0, 400000),           # the factors a fit sees
        -rng.uniform(0.0, 708.0, 200000),          # the whole normal range
        -np.ldexp(1.0, -np.arange(1, 60)),         # tiny arguments
        -np.arange(0, 708) * np.log(2.0),          # reduction boundaries n ln 2
        -(np.arange(0, 708) + 0.5) * np.log(2.0),  # and half-way between them
    ])
    ext = np.exp(x.astype(np.longdouble))
    ref = ext.astype(np.float64)
    got = _dev_exp(x)
    normal = ref >= np.finfo(np.float64).tiny
    err = (np.abs(got[normal].astype(np.longdouble) - ext[normal]) /
           np.spacing(np.abs(ref[normal])).astype(np.longdouble)).astype(np.float64)
    u = _ulps(got[normal], ref[normal])
    print(f"exp_neg: {normal.sum()} values, max error {err.max():.3f} ulp, mean "
          f"{err.mean():.4f} ulp; correctly rounded {np.mean(u == 0):.4f}")
    assert err.max() < 1.0
    assert u.max() <= 1.0


def test_exp_neg_special_values():
    x = np.array([0.0, -0.0, -1e-300, -745.2, -760.0, -1e4, np.nan])
    got = _dev_exp(x)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0
    assert 0.0 <= got[3] < 1e-320
    assert got[4] == 0.0 and got[5] == 0.0
    assert np.isnan(got[6])


def test_exp_neg_monotone():
    x = -np.linspace(0.0, 40.0, 2000001)
    y = _dev_exp(x)
    assert np.all(np.diff(y) <= 0.0)
