"""Pins taken from values the paper prints (fixtures in tests/golden/, each
with its citation): the Brio-Wu setup, the Balsara vortex and its exact
translated solution, the scale-height convention behind the stratified
box, and the scheme constants."""
import math
import os
import sys

import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import mhd
from paper_2604_12672_amd import workloads as wl

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from read import read  # noqa: E402


def primitives(w):
    """rho, v, B_cc, P of an ideal-gas workload (plain numpy, test side)."""
    U = w.U
    rho = U[0]
    v = U[1:4] / rho
    bx = 0.5 * (w.Bx + np.roll(w.Bx, -1, axis=2))
    by = 0.5 * (w.By + np.roll(w.By, -1, axis=1))
    bz = 0.5 * (w.Bz + np.roll(w.Bz, -1, axis=0))
    b = np.stack([bx, by, bz])
    P = (w.params["gamma"] - 1.0) * (U[4] - 0.5 * rho * np.sum(v * v, axis=0)
                                     - 0.5 * np.sum(b * b, axis=0))
    return rho, v, b, P


def test_brio_wu_states_match_the_paper():
    g = read("brio_wu.txt")
    w = wl.brio_wu(200, axis=0)
    assert w.params["gamma"] == g["gamma"]
    rho, v, b, P = primitives(w)
    x = (np.arange(200) + 0.5) * 2.0 / 200
    for name, xs in (("left", 1.0), ("right", 0.2)):
        i = int(np.argmin(np.abs(x - xs)))
        got = [rho[0, 0, i], v[0, 0, 0, i], v[1, 0, 0, i], b[1, 0, 0, i], P[0, 0, i]]
        np.testing.assert_allclose(got, g[name], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(w.Bx, g["B_x"], rtol=0)


def test_balsara_vortex_setup_and_rotation_count():
    g = read("balsara_vortex.txt")
    ut, bk = g["convergence_case"]
    w = wl.balsara_vortex(64, utilde=ut, beta_k=bk)
    assert tuple(w.params["lo"][:2]) == tuple(g["domain"][:1] * 2)
    assert tuple(w.params["hi"][:2]) == tuple(g["domain"][1:] * 2)
    assert w.tau == pytest.approx(10.0 * math.sqrt(2.0) / ut, rel=1e-15)
    # the rotation speed at r = 1 is u~: turns per crossing = u~ tau / (2 pi)
    assert round(ut * w.tau / (2.0 * math.pi), 2) == g["rotations_per_crossing"]
    rho, v, b, P = primitives(w)
    n = 64
    c = -5.0 + (np.arange(n) + 0.5) * 10.0 / n
    X, Y = np.meshgrid(c, c, indexing="xy")
    r2 = X * X + Y * Y
    ex = np.exp(0.5 * (1.0 - r2))
    bt = ut * math.sqrt(bk)
    np.testing.assert_allclose(rho[0], 1.0)
    np.testing.assert_allclose(v[0, 0], ut * ex * (-Y) + ut / math.sqrt(2.0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(v[1, 0], ut * ex * X + ut / math.sqrt(2.0), rtol=0, atol=1e-15)
    # face fields from the vector potential: the cell mean matches the
    # closed form to second order in dx
    dx = 10.0 / n
    np.testing.assert_allclose(b[0, 0], bt * ex * (-Y), rtol=0, atol=0.05 * bt * dx ** 2 * 10)
    np.testing.assert_allclose(b[1, 0], bt * ex * X, rtol=0, atol=0.05 * bt * dx ** 2 * 10)
    Pex = 1.0 + (0.5 * bt * bt * (1.0 - r2) - 0.5 * ut * ut) * np.exp(1.0 - r2)
    np.testing.assert_allclose(P[0], Pex, rtol=0, atol=bt * bt * dx ** 2)


def _vortex_error(n, ut, bk, frac):
    """L1 error of the oracle's vortex after frac of a crossing time against
    the exact solution (the initial vortex translated along the diagonal),
    velocity and field normalised by u~ as in the paper's convergence test."""
    w = wl.balsara_vortex(n, utilde=ut, beta_k=bk)
    o = orc.Oracle(w.params, **w.extras())
    st = w.state()
    t_end = frac * w.tau
    t = 0.0
    while t < t_end - 1e-12:
        dt = min(o.compute_dt(st, w.cfl), t_end - t)
        o.step(st, dt)
        t += dt
    shift = ut / math.sqrt(2.0) * t_end  # displacement along x and y
    c = -5.0 + (np.arange(n) + 0.5) * 10.0 / n

    def wrap(s):
        return (s + 5.0) % 10.0 - 5.0
    X, Y = np.meshgrid(wrap(c - shift), wrap(c - shift), indexing="xy")
    ex = np.exp(0.5 * (1.0 - (X * X + Y * Y)))
    vx = st["U"][1, 0] / st["U"][0, 0]
    vy = st["U"][2, 0] / st["U"][0, 0]
    e_vx = np.abs(vx - (ut * ex * (-Y) + ut / math.sqrt(2.0))).mean() / ut
    e_vy = np.abs(vy - (ut * ex * X + ut / math.sqrt(2.0))).mean() / ut
    bt = ut * math.sqrt(bk)
    bx = 0.5 * (st["Bx"][0] + np.roll(st["Bx"][0], -1, axis=1))
    e_bx = np.abs(bx - bt * ex * (-Y)).mean() / ut
    return e_vx, e_vy, e_bx


def test_balsara_vortex_translation_converges_at_second_order():
    """The oracle advects the vortex (u~ = 0.1, beta_K = 1, the paper's grid
    of models) for a quarter of a crossing time; the L1 errors against the
    exact translated vortex fall by about 4x per grid doubling."""
    e32 = _vortex_error(32, 0.1, 1.0, 0.25)
    e64 = _vortex_error(64, 0.1, 1.0, 0.25)
    for a, b in zip(e32, e64):
        assert a / b > 3.0, (e32, e64)
    assert max(e64) < 0.05, e64


def test_scale_height_convention():
    g = read("scale_heights.txt")
    assert round(math.log(g["pressure_ratio"]), 1) == g["pressure_scale_heights"]
    assert round(math.log(g["density_ratio"]), 1) == g["density_scale_heights"]
    # the stratified box spans four pressure scale heights by that count
    rho, P, _ = wl.polytrope_profile(np.array([0.0, 1.0]))
    assert math.log(P[0] / P[1]) == pytest.approx(4.0, rel=1e-14)


def test_scheme_constants_are_the_defaults():
    g = read("scheme_constants.txt")
    p = wl.base_params(4, 4, 4)
    assert p["newton_tol"] == g["newton_tol"]
    assert p["mach_cut"] == g["mach_cut"]
    d = mhd.make_desc(p)
    assert d.newton_tol == g["newton_tol"] and d.mach_cut == g["mach_cut"]
