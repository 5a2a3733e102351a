"""Accuracy of the device reciprocal and square root, through the C ABI
(`mhd_math_check`), against the correctly rounded IEEE results of numpy:
the full sequences (EOS, primitives, updates) within one ulp, those of the
FP64 flux arithmetic (one refinement step after the hardware seed) within
12 and 37 ulp.  Arguments: 2^20 seeded doubles with uniform mantissas and
exponents in [-200, 200], the powers of two 2^-60 .. 2^60 and the integers
1 .. 1000."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mhd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_12672_amd import mhd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2604_12672_amd import build
        build.build()
    m.load()
    return m


def test_device_reciprocal_and_sqrt_accuracy(mhd):
    import torch
    print("case math check, 2^20 + 1121 arguments", flush=True)
    rng = np.random.default_rng(31)
    n = 1 << 20
    x = np.ldexp(rng.uniform(1.0, 2.0, n), rng.integers(-200, 201, n))
    x = np.concatenate([x, 2.0 ** np.arange(-60, 61), np.arange(1.0, 1001.0)])
    out = mhd.math_check(torch.from_numpy(x).cuda()).cpu().numpy()
    rref, sref = 1.0 / x, np.sqrt(x)

    def ulps(got, ref):
        return np.abs(got - ref) / np.spacing(ref)

    e = [ulps(out[0], rref), ulps(out[1], rref), ulps(out[2], sref), ulps(out[3], sref)]
    print("max ulp: rcp %.2f, rcp_flux %.2f, sqrt %.2f, sqrt_flux %.2f"
          % tuple(float(v.max()) for v in e), flush=True)
    assert e[0].max() <= 1.0 and e[2].max() <= 1.0
    assert e[1].max() <= 12.0 and e[3].max() <= 37.0
    # the mean error of the one-step forms is about an ulp
    assert e[1].mean() < 2.0 and e[3].mean() < 3.0


def test_math_check_empty(mhd):
    import torch
    assert mhd.math_check(torch.empty(0, dtype=torch.float64, device="cuda")).shape == (4, 0)
