"""Pins of the oracle's EOS (Sect. 2.2, eqs. prad/erad) against closed forms
evaluated independently at 50 digits."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import workloads as wl

mp.mp.dps = 50


def _params(**kw):
    return wl.gasrad_params(2, 2, 2, **kw)


def _exact_T(rho, e, R, mu, gam, a):
    """Root of (a/rho) T^4 + R/((gamma-1) mu) T - e = 0 (the only positive one)."""
    rho, e = mp.mpf(rho), mp.mpf(e)
    cg = mp.mpf(R) / ((mp.mpf(gam) - 1) * mp.mpf(mu))
    ar = mp.mpf(a) / rho
    f = lambda t: ar * t ** 4 + cg * t - e
    hi = min(e / cg if cg > 0 else mp.inf, (e / ar) ** mp.mpf(0.25) if ar > 0 else mp.inf)
    return mp.findroot(f, (hi / 4, hi), solver="anderson")


def _e_of(p, rho, T):
    rmu = mp.mpf(p["rgas"]) / mp.mpf(p["mu"])
    return rmu * T / (mp.mpf(p["gamma"]) - 1) + mp.mpf(p["arad"]) * mp.mpf(T) ** 4 / mp.mpf(rho)


@pytest.mark.parametrize("seed", [0, 1])
def test_inversion_matches_quartic_root(seed):
    p = _params()
    o = orc.Oracle(p)
    rho_s, T_s = wl.eos_samples(40, seed=seed)
    for rho, T in zip(rho_s, T_s):
        e = float(_e_of(p, rho, mp.mpf(T)))
        Tex = _exact_T(rho, e, p["rgas"], p["mu"], p["gamma"], p["arad"])
        for guess in (T * 1.3, T * 0.5, T * 1e3, T * 1e-3):
            Tn, it, fb = o.eos_invert(rho, e, guess)
            # |de|/e < 1e-11 and e/(T c_v) <= 1 bound the relative error of T
            assert abs(Tn - float(Tex)) <= 1.0e-11 * float(Tex) * 1.01, (rho, T, guess)
            assert fb == 0


def test_inversion_limits():
    # radiation-free: T = e / C_g exactly
    p = _params(arad=0.0)
    o = orc.Oracle(p)
    cg = p["rgas"] / ((p["gamma"] - 1) * p["mu"])
    for e in (1e-3, 0.7, 12.0):
        Tn, _, _ = o.eos_invert(1.0, e, 1e6)
        assert Tn == pytest.approx(e / cg, rel=1.1e-11)
    # gas-free: T = (rho e / a)^(1/4)
    p = _params(rgas=0.0)
    p["rgas"] = 1e-300  # C_g -> 0 without a division by zero in the bracket
    o = orc.Oracle(p)
    for rho, e in ((0.1, 3.0), (10.0, 0.02)):
        Tn, _, _ = o.eos_invert(rho, e, 1e7)
        assert Tn == pytest.approx((rho * e / p["arad"]) ** 0.25, rel=1.1e-11)


def test_fallback_paths():
    p = _params()
    o = orc.Oracle(p)
    rho, T = 0.37, 2.1e6
    e = float(_e_of(p, rho, mp.mpf(T)))
    for bad in (float("nan"), -5.0, 0.0, float("inf")):
        Tn, it, fb = o.eos_invert(rho, e, bad)
        assert fb == 1
        assert Tn == pytest.approx(T, rel=1.1e-11)
    # iteration cap forces the bracketed solve
    p2 = dict(p, newton_maxit=1)
    o2 = orc.Oracle(p2)
    Tn, it, fb = o2.eos_invert(rho, e, T * 1e4)
    assert fb == 1 and Tn == pytest.approx(T, rel=1.1e-11)
    with pytest.raises(orc.OracleError):
        o.eos_invert(rho, -1.0, T)


def _entropy(p, rho, T):
    """Specific entropy of gas + radiation, s = C_g ln T - (R/mu) ln rho
    + 4 a T^3 / (3 rho) (from T ds = de + P d(1/rho))."""
    rmu = mp.mpf(p["rgas"]) / mp.mpf(p["mu"])
    cg = rmu / (mp.mpf(p["gamma"]) - 1)
    return cg * mp.log(T) - rmu * mp.log(rho) + 4 * mp.mpf(p["arad"]) * T ** 3 / (3 * rho)


def _P(p, rho, T):
    rmu = mp.mpf(p["rgas"]) / mp.mpf(p["mu"])
    return rho * rmu * T + mp.mpf(p["arad"]) * T ** 4 / 3


@pytest.mark.parametrize("rho,T", [(1e-2, 1e5), (1.0, 3e6), (0.05, 1e8), (30.0, 2e7)])
def test_sound_speed_is_adiabatic_derivative(rho, T):
    """c_s^2 = (dP/drho)_s along the exact adiabat, by a high-precision central
    difference."""
    p = _params()
    o = orc.Oracle(p)
    P, e, cv, cs2 = o.eos_thermo(rho, T)
    r0, T0 = mp.mpf(rho), mp.mpf(T)
    s0 = _entropy(p, r0, T0)
    h = mp.mpf("1e-12")

    def T_on_adiabat(r):
        return mp.findroot(lambda t: _entropy(p, r, t) - s0, T0)

    rp, rm = r0 * (1 + h), r0 * (1 - h)
    dPdrho = (_P(p, rp, T_on_adiabat(rp)) - _P(p, rm, T_on_adiabat(rm))) / (rp - rm)
    assert cs2 == pytest.approx(float(dPdrho), rel=1e-12)
    assert P == pytest.approx(float(_P(p, r0, T0)), rel=1e-14)
    assert e == pytest.approx(float(_e_of(p, rho, T0)), rel=1e-14)


def test_gamma_limits():
    """gamma_c -> gamma for a gas without radiation, -> 4/3 for radiation."""
    p = _params()
    o = orc.Oracle(dict(p, arad=0.0))
    P, e, cv, cs2 = o.eos_thermo(1.0, 1e6)
    assert cs2 * 1.0 / P == pytest.approx(5.0 / 3.0, rel=1e-14)
    assert P / (1.0 * e) + 1 == pytest.approx(5.0 / 3.0, rel=1e-14)
    o = orc.Oracle(dict(p, rgas=1e-300))
    P, e, cv, cs2 = o.eos_thermo(1.0, 1e7)
    assert cs2 / P == pytest.approx(4.0 / 3.0, rel=1e-12)
    assert P / e + 1 == pytest.approx(4.0 / 3.0, rel=1e-12)


def test_newton_steps_against_guess_error():
    """Newton's quadratic convergence in the inversion (Sect. 2.2): the steps
    it takes fall as the guess improves, and a guess within 1e-8 dex
    converges in one step.  The table is what a learned guess would have
    to reach to save steps (the polish of a BF16 network, about 3e-3 dex,
    takes about 2.2 steps on average)."""
    p = _params()
    o = orc.Oracle(p)
    rho_s, T_s = wl.eos_samples(300, seed=7)
    rng = np.random.default_rng(7)
    sign = rng.choice((-1.0, 1.0), size=len(rho_s))
    e_s = [o.eos_thermo(r, t)[1] for r, t in zip(rho_s, T_s)]
    means = {}
    for dex in (1e-1, 1e-2, 3e-3, 1e-4, 1e-6, 1e-8):
        its = []
        for r, e, t, sg in zip(rho_s, e_s, T_s, sign):
            Tn, it, fb = o.eos_invert(r, e, t * 10.0 ** (sg * dex))
            assert fb == 0
            assert abs(Tn - t) <= 2e-11 * t
            its.append(it)
        means[dex] = float(np.mean(its))
    print({k: round(v, 2) for k, v in means.items()})
    vals = [means[d] for d in sorted(means, reverse=True)]
    assert all(a >= b for a, b in zip(vals, vals[1:])), means
    assert means[1e-8] == 1.0
    assert means[3e-3] >= 2.0
