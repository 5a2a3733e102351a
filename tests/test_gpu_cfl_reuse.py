"""The first stage of a step takes what the CFL kernel computed on the same
state: the thermal pressure for the shock detector (flattening on) and the
converged temperatures (gas + radiation).  These tests drive that path
through `mhd_advance` (dt from the device each step) and check it against
the oracle's own CFL-and-step loop, for the ideal gas and gas + radiation,
the previous-step and the learned guess, FP64 and split precision; and that
loading another state between the CFL call and the step discards what the
CFL kernel left.

Tolerances are those of the host-dt parity tests (FP64 rel L2 1e-10, 1e-9
with the gas + radiation Newton tolerance; split 1e-5): the device dt
agrees with the oracle's to about 1e-12."""
import math
import os

import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import eos_mlp
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


def rel_errors(out, ref):
    """rel L2 per field; momentum and field components against their
    vector's norm."""
    vm = sum(norm2(ref["U"][c]) for c in (1, 2, 3))
    vb = sum(norm2(ref[k]) for k in ("Bx", "By", "Bz"))
    errs = {"rho": math.sqrt(norm2(out["U"][0] - ref["U"][0]) / norm2(ref["U"][0])),
            "E": math.sqrt(norm2(out["U"][4] - ref["U"][4]) / norm2(ref["U"][4]))}
    for c in (1, 2, 3):
        errs[f"m{c}"] = math.sqrt(norm2(out["U"][c] - ref["U"][c]) / vm)
    for k in ("Bx", "By", "Bz"):
        errs[k] = math.sqrt(norm2(out[k] - ref[k]) / vb)
    return errs


def _with(w, **kw):
    return wl.Workload(w.name, dict(w.params, **kw), w.U, w.Bx, w.By, w.Bz, T=w.T,
                       bg_cc=w.bg_cc, bg_fz=w.bg_fz, heat=w.heat, fmodes=w.fmodes, cfl=w.cfl)


CASES = [
    # name, shape, bcz, eos, flatten, recon, rk, guess, precision, tol
    ("ideal-flat-vl", (20, 17, 13), 0, wl.EOS_IDEAL, 1, orc.RECON_VANLEER, 2, "prev", 0, 1e-10),
    ("ideal-flat-pph-split", (19, 15, 14), 1, wl.EOS_IDEAL, 1, orc.RECON_PPH, 3, "prev", 1, 1e-5),
    ("gasrad-flat-prevT", (12, 11, 10), 0, wl.EOS_GASRAD, 1, orc.RECON_PPH, 3, "prev", 0, 1e-9),
    ("gasrad-prevT", (14, 12, 10), 1, wl.EOS_GASRAD, 0, orc.RECON_VANLEER, 2, "prev", 0, 1e-9),
    ("gasrad-flat-learned", (18, 15, 12), 1, wl.EOS_GASRAD, 1, orc.RECON_VANLEER, 2, "mlp", 0,
     1e-9),
    ("gasrad-learned", (18, 15, 12), 1, wl.EOS_GASRAD, 0, orc.RECON_PPH, 3, "mlp", 0, 1e-9),
    ("gasrad-learned-split", (18, 15, 12), 1, wl.EOS_GASRAD, 0, orc.RECON_VANLEER, 2, "mlp", 1,
     1e-5),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_advance_matches_oracle_cfl_loop(mhd, case):
    name, shape, bcz, eos, flatten, recon, rk, guess, precision, tol = case
    print(f"case {name} {shape} bcz={bcz}", flush=True)
    w = wl.smooth_box(*shape, bcz=bcz, eos=eos, blast=(10.0, 0.3) if flatten else None)
    w = _with(w, flatten=flatten, recon=recon, rk_order=rk)
    o = orc.Oracle(w.params, **w.extras())
    ref = w.state()
    nsteps = 3
    for _ in range(nsteps):
        o.step(ref, o.compute_dt(ref, w.cfl))
    kw = dict(precision=precision)
    if guess == "mlp":
        kw["eos_guess"] = mhd.GUESS_MLP
    g = mhd.Grid(w.params, **kw)
    g.load(w, mlp=eos_mlp.MLPGuess.load() if guess == "mlp" else None)
    g.advance(w.cfl, nsteps)
    out = g.get_state()
    flags = g.shock_flags() if flatten else None
    diag = g.diagnostics()
    g.close()
    errs = rel_errors(out, ref)
    assert all(v <= tol for v in errs.values()), errs
    assert diag["divb_max"] < 1e-12
    if flatten and precision == 0:
        assert np.array_equal(flags, o.shock_flags(ref))
    if eos == wl.EOS_GASRAD:
        assert diag["fallbacks"] == 0


@pytest.mark.parametrize("eos,guess", [(wl.EOS_IDEAL, "prev"), (wl.EOS_GASRAD, "prev"),
                                       (wl.EOS_GASRAD, "mlp")])
def test_new_state_discards_cfl_results(mhd, eos, guess):
    """CFL on a blast state, then a smooth state loaded and stepped with
    that dt: the step must run on the smooth state's own pressure and
    temperatures.  A detector threshold of 4 makes the two states' flags
    differ in most cells, so a step on the blast state's pressures would
    switch reconstruction and solver in the wrong cells."""
    print(f"case discard eos={eos} guess={guess}", flush=True)
    shape = (16, 14, 12)
    a = _with(wl.smooth_box(*shape, eos=eos, blast=(10.0, 0.3)), flatten=1, eps_sf=4.0,
              recon=orc.RECON_PPH, rk_order=3)
    b = _with(wl.smooth_box(*shape, eos=eos, seed=5), flatten=1, eps_sf=4.0,
              recon=orc.RECON_PPH, rk_order=3)
    kw = {"eos_guess": mhd.GUESS_MLP} if guess == "mlp" else {}
    g = mhd.Grid(a.params, **kw)
    g.load(a, mlp=eos_mlp.MLPGuess.load() if guess == "mlp" else None)
    dt = 0.5 * g.compute_dt(a.cfl)
    g.load(b)  # the network stays: only the state changes
    g.step(dt)
    out = g.get_state()
    g.close()
    o = orc.Oracle(b.params, **b.extras())
    ref = b.state()
    fa = o.shock_flags(a.state())
    fb = o.shock_flags(ref)
    assert (fa != fb).sum() > fa.size // 4
    o.step(ref, dt)
    errs = rel_errors(out, ref)
    assert all(v <= 1e-9 for v in errs.values()), errs
