"""Parity of mhd_diagnostics with the oracle and with exact sums.

div B of eq. divb (Sect. 2.4, constrained transport) is the oracle's
orc_divb of the face field the library holds; the conserved totals and the
magnetic flux through the plane x_{-1/2} (Sect. 2.3, the conservation the
finite-volume form eq. fv guarantees) are exactly rounded sums (math.fsum)
of the arrays mhd_get_state returns.  The library reports

  divb_max  = max_cells |div B| dx_min / max |B_face|
  divb_l2   = sqrt(mean_cells (div B dx_min)^2) / max |B_face|
  bface_max = max |B_face| over the stored faces (wall planes included)
  total[f]  = sum over cells of U[f]
  bflux_x0  = sum over (j, k) of B_x on the face x_{-1/2}

Bounds.  div B of one cell is a sum of three differences of faces scaled
by 1/dx_s; the kernel multiplies by the stored reciprocal where the oracle
divides, so each cell value is within 4 eps (|d_x| + |d_y| + |d_z|) of the
exact one, d_s the three terms; the max is within the largest such bound,
the L2 norm within the L2 norm of the bounds.  The sums are reduced in a
fixed order in blocks (a tree of 256 and a grid stride per block, then a
long-double sum of the block partials), so each is within
(8 + passes + 2) eps sum |x| of the exact sum; 1e-14 sum |x| covers every
grid here.  The face maximum is exact."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import workloads as wl

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


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


def _dx(p):
    return [(p["hi"][a] - p["lo"][a]) / (p["nx"], p["ny"], p["nz"])[a] for a in range(3)]


def _terms(p, st):
    """The three terms of div B per cell (numpy, for the rounding bound)."""
    Bx, By, Bz = st["Bx"], st["By"], st["Bz"]
    dx, dy, dz = _dx(p)
    tx = (np.roll(Bx, -1, axis=2) - Bx) / dx
    ty = (np.roll(By, -1, axis=1) - By) / dy
    if p["bcz"] == wl.BC_REFLECT:
        tz = (Bz[1:] - Bz[:-1]) / dz
    else:
        tz = (np.roll(Bz, -1, axis=0) - Bz) / dz
    return tx, ty, tz


def check_diag(p, st, diag):
    o = orc.Oracle(p)
    dmin = min(_dx(p))
    bmax = max(float(np.max(np.abs(st[k]))) for k in ("Bx", "By", "Bz"))
    assert diag["bface_max"] == bmax
    d = o.divb(st) * dmin
    tx, ty, tz = _terms(p, st)
    bound = 4 * EPS * (np.abs(tx) + np.abs(ty) + np.abs(tz)) * dmin
    ref_max = float(np.max(np.abs(d))) / bmax
    ref_l2 = math.sqrt(float(np.mean(d * d))) / bmax
    assert abs(diag["divb_max"] - ref_max) <= 2 * float(np.max(bound)) / bmax, (
        diag["divb_max"], ref_max)
    assert abs(diag["divb_l2"] - ref_l2) <= (
        2 * math.sqrt(float(np.mean(bound * bound))) / bmax + 1e-15 * ref_l2), (
        diag["divb_l2"], ref_l2)
    U = st["U"]
    for f in range(5):
        x = U[f].ravel()
        exact = math.fsum(x)
        assert abs(diag["total"][f] - exact) <= 1e-14 * math.fsum(np.abs(x)) + 1e-300, (
            f, diag["total"][f], exact)
    x = st["Bx"][:, :, 0].ravel()
    exact = math.fsum(x)
    assert abs(diag["bflux_x0"] - exact) <= 1e-14 * math.fsum(np.abs(x)) + 1e-300
    return ref_max, ref_l2


@pytest.mark.parametrize("shape,bcz", [((80, 70, 61), 0), ((33, 29, 17), 1), ((7, 1, 5), 0)])
def test_random_face_field(mhd, shape, bcz):
    """A face field of independent random values (div B of order |B|/dx in
    every cell) on ragged grids; the larger one spans several grid-stride
    passes of the reduction, the walled one has zeroed wall planes."""
    nx, ny, nz = shape
    print(f"case random face field {shape} bcz={bcz}", flush=True)
    w = wl.smooth_box(nx, ny, nz, bcz=bcz)
    rng = np.random.default_rng(31)
    st = w.state()
    for k in ("Bx", "By", "Bz"):
        st[k] = st[k] + rng.uniform(-1.0, 1.0, size=st[k].shape)
    st["U"][1:4] += rng.uniform(-0.5, 0.5, size=st["U"][1:4].shape)
    with mhd.Grid(w.params) as g:
        g.set_state(st["U"], st["Bx"], st["By"], st["Bz"])
        held = g.get_state()
        diag = g.diagnostics()
    if bcz == wl.BC_REFLECT:
        assert np.all(held["Bz"][0] == 0.0) and np.all(held["Bz"][-1] == 0.0)
        assert np.array_equal(held["Bz"][1:-1], st["Bz"][1:-1])
    ref_max, ref_l2 = check_diag(w.params, held, diag)
    # order-one divergence: the relative agreement the bounds imply
    assert diag["divb_max"] == pytest.approx(ref_max, rel=1e-14)
    assert diag["divb_l2"] == pytest.approx(ref_l2, rel=1e-14)
    assert ref_max > 0.1


def _exact_divb_max(p, st):
    """max |div B| dx_min / max |B_face| in exact rational arithmetic on the
    stored doubles (the box edges are exact in binary here)."""
    nz, ny, nx = st["Bx"].shape
    L = [Fraction(p["hi"][a]) - Fraction(p["lo"][a]) for a in range(3)]
    n = (nx, ny, nz)
    dx = [L[a] / n[a] for a in range(3)]
    dmin = min(dx)
    Bx = [[[Fraction(v) for v in row] for row in pl] for pl in st["Bx"]]
    By = [[[Fraction(v) for v in row] for row in pl] for pl in st["By"]]
    Bz = [[[Fraction(v) for v in row] for row in pl] for pl in st["Bz"]]
    refl = p["bcz"] == wl.BC_REFLECT
    m = Fraction(0)
    for k in range(nz):
        kp = k + 1 if refl else (k + 1) % nz
        for j in range(ny):
            jp = (j + 1) % ny
            for i in range(nx):
                ip = (i + 1) % nx
                d = ((Bx[k][j][ip] - Bx[k][j][i]) / dx[0] + (By[k][jp][i] - By[k][j][i]) / dx[1]
                     + (Bz[kp][j][i] - Bz[k][j][i]) / dx[2])
                m = max(m, abs(d))
    bmax = max(float(np.max(np.abs(st[k]))) for k in ("Bx", "By", "Bz"))
    return float(m * dmin / Fraction(bmax))


@pytest.mark.parametrize("precision", [0, 1])
def test_ct_evolved_state(mhd, precision):
    """A state advanced by the constrained-transport update (the stratified
    box with walls, 6 steps): div B stays at round-off, and the reported
    value is the exact divergence of the stored faces to within the
    rounding of its own evaluation."""
    print(f"case ct-evolved stratified 16x16x20 prec={precision}", flush=True)
    w = wl.stratified_box(16, nz=20)
    with mhd.Grid(w.params, precision=precision) as g:
        g.load(w)
        for _ in range(6):
            g.step(g.compute_dt(w.cfl))
        held = g.get_state()
        diag = g.diagnostics()
    check_diag(w.params, held, diag)
    exact = _exact_divb_max(w.params, held)
    tx, ty, tz = _terms(w.params, held)
    bmax = diag["bface_max"]
    bound = 4 * EPS * float(np.max(np.abs(tx) + np.abs(ty) + np.abs(tz))) * min(_dx(w.params))
    assert abs(diag["divb_max"] - exact) <= 2 * bound / bmax, (diag["divb_max"], exact)
    assert diag["divb_max"] < 1e-12 and exact < 1e-12
