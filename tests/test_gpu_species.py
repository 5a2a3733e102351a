"""Passive species (Sect. 2.9) on the GPU against the oracle, through the C
ABI: the partial densities rho X_l after several steps with van Leer +
SSP-RK2 and PPH (limited parabola for the fractions) + SSP-RK3, with and
without shock flattening, periodic and walled boxes, FP64 and split
precision, 1 to 12 species; the species masses add up to the density.

Tolerances: rel L2 per species <= 1e-10 (FP64), <= 1e-5 (split): the
species fluxes are the stage's mass fluxes times fractions of the FP64
stage input, so they follow the mass flux's precision.  The sum of the
species masses equals the density to FP64 rounding in both modes (the
same mass flux carries both)."""
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


def rel_l2(a, b):
    den = math.sqrt(float(np.sum(b * b)))
    return math.sqrt(float(np.sum((a - b) ** 2))) / den


def _case(shape, bcz, ns, blast, **kw):
    w = wl.smooth_box(*shape, bcz=bcz, blast=(4.0, 0.3) if blast else None)
    w = wl.add_species(w, ns)
    w.params = dict(w.params, **kw)
    return w


def run_pair(mhd, w, nsteps, precision=0):
    print(f"case {w.name} {w.shape} ns={w.params['nspecies']} recon={w.params.get('recon')} "
          f"rk{w.params.get('rk_order')} flat={w.params.get('flatten')} prec={precision}",
          flush=True)
    o = orc.Oracle(w.params, **w.extras())
    ref = w.state()
    dts = []
    for _ in range(nsteps):
        dt = o.compute_dt(ref, w.cfl)
        o.step(ref, dt)
        dts.append(dt)
    g = mhd.Grid(w.params, precision=precision)
    g.load(w)
    for dt in dts:
        g.step(dt)
    out = g.get_state()
    X = g.get_species()
    g.close()
    return out, X, ref


CASES = [((20, 17, 13), 0, 1, False, dict()),
         ((19, 15, 14), 1, 3, False, dict(recon=orc.RECON_PPH, rk_order=3)),
         ((20, 17, 13), 0, 12, True, dict(recon=orc.RECON_PPH, rk_order=3, flatten=1)),
         ((19, 15, 14), 1, 5, True, dict(flatten=1)),
         ((1, 24, 9), 0, 4, False, dict(recon=orc.RECON_PPH)),
         # walls with three z segments of the species kernel (32, 32, 6
         # planes), a ragged y tile and the largest species count
         ((18, 9, 70), 1, 16, True, dict(recon=orc.RECON_PPH, rk_order=3, flatten=1)),
         # one cell along y; two z segments
         ((33, 1, 40), 0, 8, False, dict()),
         # one cell along z
         ((17, 10, 1), 0, 6, False, dict(rk_order=3))]


@pytest.mark.parametrize("shape,bcz,ns,blast,kw", CASES)
@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-5)])
def test_species_match_oracle(mhd, shape, bcz, ns, blast, kw, precision, tol):
    w = _case(shape, bcz, ns, blast, **kw)
    out, X, ref = run_pair(mhd, w, 3, precision)
    for l in range(ns):
        e = rel_l2(X[l], ref["U"][5 + l])
        assert e <= tol, (l, e)
    assert rel_l2(out["U"][0], ref["U"][0]) <= tol
    np.testing.assert_allclose(X.sum(axis=0), out["U"][0], rtol=1e-13, atol=0)


def test_species_across_tiles_and_segments(mhd):
    """96^3 blast box with 12 species, PPH + SSP-RK3 + flattening: several
    tiles (ragged last), z segments, one step against the full oracle."""
    w = _case((96, 96, 96), 0, 12, True, recon=orc.RECON_PPH, rk_order=3, flatten=1)
    out, X, ref = run_pair(mhd, w, 1)
    for l in range(12):
        assert rel_l2(X[l], ref["U"][5 + l]) <= 1e-10, l
    np.testing.assert_allclose(X.sum(axis=0), out["U"][0], rtol=1e-13, atol=0)


def test_species_error_paths(mhd):
    w = wl.add_species(wl.smooth_box(8, 8, 8), 2)
    g = mhd.Grid(w.params)
    g.set_state(np.ascontiguousarray(w.U[:5]), w.Bx, w.By, w.Bz)
    with pytest.raises(mhd.MHDError):
        g.step(1e-3)  # species not set
    with pytest.raises(mhd.MHDError):
        g.get_species()
    g.set_species(w.U[5:])
    g.step(1e-3)
    g.close()
    w0 = wl.smooth_box(8, 8, 8)
    g0 = mhd.Grid(w0.params)
    g0.load(w0)
    with pytest.raises(mhd.MHDError):
        g0.set_species(np.ones((0, 8, 8, 8)))
    g0.close()
