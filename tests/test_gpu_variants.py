"""The stage kernel is compiled twice: without and with the code of the
optional features (forcing modes, shock-flattening flags, species mass
fluxes).  Where a feature is present but changes nothing, the two variants
must give the same fluid state bit for bit:
- forcing modes of zero amplitude (the sources add exact zeros),
- flattening with a detector threshold no cell reaches (no flags: every
  face takes LHLLD, every cell its own reconstruction),
- passive species (the fluid does not see them).
Compared with numpy's array_equal, for which -0.0 equals 0.0."""
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


def run(mhd, w, dts, precision, species=None):
    g = mhd.Grid(w.params, precision=precision)
    g.load(w)
    if species is not None:
        g.set_species(species)
    for dt in dts:
        g.step(dt)
    out = g.get_state()
    g.close()
    return out


def cfl_dt(w, cfl=0.3):
    """dt of the initial state at the given CFL number (the oracle's)."""
    return orc.Oracle(w.params, **w.extras()).compute_dt(w.state(), cfl)


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("U", "Bx", "By", "Bz"))


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_forcing_matches_no_forcing(mhd, precision):
    print(f"case zero forcing prec={precision}", flush=True)
    w = wl.smooth_box(20, 17, 13, bcz=1)
    dts = [cfl_dt(w)] * 3
    a = run(mhd, w, dts, precision)
    # forcing modes of zero amplitude (every wavenumber kind of the basis)
    zero = [[kx, ky, kz, 0.0, 0.0, 0.0, 0.3] for kx, ky, kz in
            ((1, 0, 0), (0, 1, 1), (1, -1, -2), (2, 1, 2), (0, 0, -1))]
    wf = wl.Workload(w.name, w.params, w.U, w.Bx, w.By, w.Bz, bg_cc=w.bg_cc, bg_fz=w.bg_fz,
                     fmodes=np.array(zero), cfl=w.cfl)
    b = run(mhd, wf, dts, precision)
    assert same(a, b)


@pytest.mark.parametrize("precision,recon,rk", [(0, orc.RECON_PPH, 3), (1, orc.RECON_VANLEER, 2)])
def test_flattening_without_flags_matches_off(mhd, precision, recon, rk):
    print(f"case flattening without flags prec={precision} recon={recon}", flush=True)
    w = wl.smooth_box(19, 15, 14, bcz=1)
    w.params = dict(w.params, recon=recon, rk_order=rk)
    dts = [cfl_dt(w)] * 2
    a = run(mhd, w, dts, precision)
    wflat = wl.Workload(w.name, dict(w.params, flatten=1, eps_sf=1e30), w.U, w.Bx, w.By, w.Bz,
                        bg_cc=w.bg_cc, bg_fz=w.bg_fz, cfl=w.cfl)
    g = mhd.Grid(wflat.params, precision=precision)
    g.load(wflat)
    assert g.shock_flags().sum() == 0
    g.close()
    b = run(mhd, wflat, dts, precision)
    assert same(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_species_do_not_change_the_fluid(mhd, precision):
    print(f"case species vs none prec={precision}", flush=True)
    w = wl.smooth_box(18, 16, 12)
    w.params = dict(w.params, recon=orc.RECON_PPH, rk_order=3)
    dts = [cfl_dt(w)] * 2
    a = run(mhd, w, dts, precision)
    ws = wl.add_species(w, 3)
    b = run(mhd, ws, dts, precision)
    assert same(a, b)
