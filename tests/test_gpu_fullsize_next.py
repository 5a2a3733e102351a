"""Parity at the benchmark's full sizes for the shock flattening, the
passive species and the RKL2 thermal diffusion, in the launch
configuration the benchmark times, against full-grid oracle runs.

- 256^3 blast box (PPH + SSP-RK3 + flattening): the flags of the input and
  of the state after one step bit for bit, the state to rel L2 1e-10.
- 256^3 stratified box with 12 species (PPH + SSP-RK3): one step, every
  species to rel L2 1e-10, the species masses adding up to the density.
- 256^3 gas + radiation box, one RKL2 super step of five stages in both
  forms: E and T to rel L2 1e-9 (the Newton tolerance argument of the
  small-grid diffusion tests).

Momentum and field components are measured against their vector's norm
(components that vanish in exact arithmetic carry rounding noise only)."""
import math
import os

import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import workloads as wl

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


def norm2(a):
    return float(np.sum(a * a))


def state_errors(out, ref):
    vm = sum(norm2(ref["U"][c]) for c in (1, 2, 3))
    vb = sum(norm2(ref[k]) for k in ("Bx", "By", "Bz"))
    errs = {}
    for name, a, b, den in (("rho", out["U"][0], ref["U"][0], norm2(ref["U"][0])),
                            ("m_x", out["U"][1], ref["U"][1], vm),
                            ("m_y", out["U"][2], ref["U"][2], vm),
                            ("m_z", out["U"][3], ref["U"][3], vm),
                            ("E", out["U"][4], ref["U"][4], norm2(ref["U"][4])),
                            ("Bx", out["Bx"], ref["Bx"], vb), ("By", out["By"], ref["By"], vb),
                            ("Bz", out["Bz"], ref["Bz"], vb)):
        errs[name] = math.sqrt(norm2(a - b) / den)
    return errs


def test_blast_256_flags_and_step(mhd):
    print("case blast 256^3 PPH RK3 flattening", flush=True)
    w = wl.smooth_box(256, 256, 256, blast=(10.0, 0.25))
    w.params = dict(w.params, flatten=1, recon=orc.RECON_PPH, rk_order=3)
    o = orc.Oracle(w.params, **w.extras())
    ref = w.state()
    f0 = o.shock_flags(ref)
    dt = o.compute_dt(ref, 0.4)
    o.step(ref, dt)
    f1 = o.shock_flags(ref)
    g = mhd.Grid(w.params)
    g.load(w)
    assert np.array_equal(g.shock_flags(), f0)
    g.step(dt)
    out = g.get_state()
    g1 = g.shock_flags()
    g.close()
    assert 0.001 < f0.mean() < 0.5
    assert np.array_equal(g1, f1)
    errs = state_errors(out, ref)
    assert all(v <= 1e-10 for v in errs.values()), errs


def test_species_256_one_step(mhd):
    print("case 12 species 256^3 PPH RK3", flush=True)
    w0 = wl.stratified_box(256, cfl=0.8)
    w0.params = dict(w0.params, recon=orc.RECON_PPH, rk_order=3)
    w = wl.add_species(w0, 12)
    o = orc.Oracle(w.params, **w.extras())
    ref = w.state()
    dt = o.compute_dt(ref, w.cfl)
    o.step(ref, dt)
    g = mhd.Grid(w.params)
    g.load(w)
    g.step(dt)
    out = g.get_state()
    X = g.get_species()
    g.close()
    for l in range(12):
        e = math.sqrt(norm2(X[l] - ref["U"][5 + l]) / norm2(ref["U"][5 + l]))
        assert e <= 1e-10, (l, e)
    np.testing.assert_allclose(X.sum(axis=0), out["U"][0], rtol=1e-13, atol=0)


@pytest.mark.parametrize("mode", [orc.DIFF_EINT, orc.DIFF_TEMP])
def test_rkl2_256_super_step(mhd, mode):
    print(f"case rkl2 256^3 mode={mode}", flush=True)
    w = wl.config(3, 256)
    op = orc.opacity(0.2, alpha=1.0, beta=-3.5)
    o = orc.Oracle(w.params, **w.extras())
    ref = w.state()
    rho = ref["U"][0]
    dtp = o.parabolic_dt(rho, ref["T"], op)
    g = mhd.Grid(w.params)
    g.load(w)
    g.set_opacity(0.2, alpha=1.0, beta=-3.5)
    assert g.parabolic_dt() == pytest.approx(dtp, rel=1e-9)
    dt = 6.0 * dtp
    o.diffuse(ref, dt, 5, op, mode=mode)
    g.diffuse(dt, 5, mode)
    out = g.get_state(with_T=True)
    g.close()
    eE = math.sqrt(norm2(out["U"][4] - ref["U"][4]) / norm2(ref["U"][4]))
    eT = math.sqrt(norm2(out["T"] - ref["T"]) / norm2(ref["T"]))
    assert eE <= 1e-9 and eT <= 1e-9, (eE, eT)
    # only the energy changes
    np.testing.assert_array_equal(out["U"][:4], w.U[:4])
