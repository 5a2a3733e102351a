"""The learned EOS guess (offline part): its training samples come from the
same forward EOS as the oracle's, the committed BF16 network reproduces T
from (rho, e) to a few 1e-3 dex, and the oracle's Newton polishes its guess
within the learned-mode cap without the bracketed fallback."""
import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import eos_mlp
from paper_2604_12672_amd import workloads as wl


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -2.5, 3.0e-3],
                 dtype=np.float32)
    r = eos_mlp.bf16_round(x)
    # 1 + 2^-9 is a tie -> even (1.0); 1 + 3*2^-9 rounds up to 1 + 2^-7
    np.testing.assert_array_equal(r[:4], np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0], np.float32))
    assert r[4] == -2.5
    assert abs(r[5] / 3.0e-3 - 1) < 2 ** -8


def test_samples_match_oracle_eos():
    p = wl.gasrad_params(2, 2, 2)
    o = orc.Oracle(p)
    rho, e, T = eos_mlp.sample(p, 200, seed=3)
    for r, ee, t in zip(rho, e, T):
        P, eo, cv, cs2 = o.eos_thermo(r, t)
        assert ee == pytest.approx(eo, rel=1e-14)


def test_committed_model_accuracy_and_polish():
    p = wl.gasrad_params(2, 2, 2)
    m = eos_mlp.MLPGuess.load()
    rho, e, T = eos_mlp.sample(p, 20000, seed=99)
    err = np.abs(m.predict_log10T(rho, e) - np.log10(T))
    assert err.mean() < 0.01 and err.max() < 0.06, (err.mean(), err.max())
    o = orc.Oracle(dict(p, newton_maxit=8))
    T0 = m.predict_T(rho[:500], e[:500])
    for r, ee, t, g in zip(rho[:500], e[:500], T[:500], T0):
        Tn, it, fb = o.eos_invert(r, ee, g)
        assert fb == 0 and it <= 8
        assert Tn == pytest.approx(t, rel=1.01e-11)
