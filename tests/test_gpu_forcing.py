"""Forcing from Fourier modes on the GPU against the oracle.

The library takes the driven-turbulence forcing as its 32 Fourier modes
and evaluates the acceleration of every cell inside the stage kernel (per
column coefficients of a z basis, summed once on the host); the oracle
evaluates the same modes term by term at the cell centres (orc_forcing,
pinned by the FFT of its field).  The turbulence box (gas + radiation,
rms Mach 3, beta 1) at a small size steps with both, in FP64 (rel L2 1e-9:
the inversion's tolerance) and in the precision split with the learned
guess (1e-5), and on ragged and walled smooth boxes with random modes."""
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


def rel_l2(a, b):
    den = math.sqrt(float(np.sum(b * b)))
    return math.sqrt(float(np.sum((a - b) ** 2))) / den if den > 0 else math.sqrt(float(np.sum(a * a)))


def run_pair(mhd, w, nsteps, precision, mlp=None):
    o = orc.Oracle(w.params, **w.extras())
    ref = w.state()
    dts = []
    for _ in range(nsteps):
        dt = o.compute_dt(ref, w.cfl)
        o.step(ref, dt)
        dts.append(dt)
    guess = mhd.GUESS_MLP if mlp is not None else mhd.GUESS_PREV_T
    with mhd.Grid(w.params, precision=precision, eos_guess=guess) as g:
        g.load(w, mlp=mlp)
        for dt in dts:
            g.step(dt)
        out = g.get_state()
        diag = g.diagnostics()
    return out, ref, diag


def check(out, ref, tol, what):
    errs = {}
    for key, c in (("U", 0), ("U", 1), ("U", 2), ("U", 3), ("U", 4), ("Bx", None), ("By", None),
                   ("Bz", None)):
        a = out[key] if c is None else out[key][c]
        b = ref[key] if c is None else ref[key][c]
        errs[f"{key}{'' if c is None else c}"] = rel_l2(a, b)
    print(what, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert all(v <= tol for v in errs.values()), (what, errs)


@pytest.mark.parametrize("precision,learned,tol", [(0, False, 1e-9), (1, True, 1e-5)])
def test_turbulence_forcing_modes(mhd, precision, learned, tol):
    print(f"case forced turbulence 24^3 prec={precision} learned={learned}", flush=True)
    w = wl.turbulence_box(24)
    assert w.fmodes.shape == (32, 7)
    mlp = eos_mlp.MLPGuess.load() if learned else None
    out, ref, diag = run_pair(mhd, w, 3, precision, mlp)
    check(out, ref, tol, f"turbulence prec={precision}")
    assert diag["divb_max"] < 1e-12
    # the forcing acts: without it the momentum differs by far more
    w0 = wl.turbulence_box(24, forcing=False)
    out0, _, _ = run_pair(mhd, w0, 3, precision, mlp)
    assert rel_l2(out0["U"][1], ref["U"][1]) > 100 * tol


@pytest.mark.parametrize("shape,bcz", [((21, 13, 9), 1), ((10, 17, 12), 0)])
def test_random_modes_on_smooth_boxes(mhd, shape, bcz):
    """Random modes (|k_x|, |k_y| up to 3, every |k_z| <= 2) on ragged boxes
    with walls and periodic; FP64 and split."""
    rng = np.random.default_rng(23)
    modes = []
    for _ in range(9):
        k = [int(rng.integers(-3, 4)), int(rng.integers(-3, 4)), int(rng.integers(-2, 3))]
        modes.append(k + list(rng.normal(size=3) * 0.5) + [rng.uniform(0, 2 * np.pi)])
    for precision, tol in ((0, 1e-11), (1, 1e-5)):
        w = wl.smooth_box(*shape, bcz=bcz)
        w.fmodes = np.array(modes)
        print(f"case random modes {shape} bcz={bcz} prec={precision}", flush=True)
        out, ref, diag = run_pair(mhd, w, 3, precision)
        check(out, ref, tol, f"smooth {shape} prec={precision}")
        assert diag["divb_max"] < 1e-12


def test_mode_checks(mhd):
    w = wl.smooth_box(8, 8, 8)
    with mhd.Grid(w.params) as g:
        for bad in ([[1, 0, 3, 1, 0, 0, 0]], [[0.5, 0, 0, 1, 0, 0, 0]],
                    [[1, 0, 0, np.nan, 0, 0, 0]]):
            with pytest.raises(mhd.MHDError) as e:
                g.set_sources(None, np.array(bad, dtype=float))
            assert e.value.code == -1
