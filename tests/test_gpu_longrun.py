"""The target's accuracy statement over 50 steps on the workloads with the
learned EOS guess: the FP32+learned-EOS step against the FP64 oracle on
the oracle's own dt sequence, every field within rel L2 1e-5 and div B at
round-off, on the gas + radiation box (config 3's recipe at 64^3) and the
forced Mach-3 turbulence box (config 4's recipe at 48^3: 32 forcing modes,
beta 1), sizes at which the host oracle takes seconds.  The FP64 path on
the same runs stays within 1e-10 (these boxes have no background, so the
oracle's own rounding floor of the stratified boxes does not arise;
measured 2e-15).  Measured split + learned: 1.2e-7 (gas + radiation,
momentum) and 4.5e-8 (turbulence)."""
import math
import os

import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import eos_mlp
from paper_2604_12672_amd import workloads as wl

pytestmark = pytest.mark.gpu
FIELDS = (("U", 0), ("U", 1), ("U", 2), ("U", 3), ("U", 4), ("Bx", None), ("By", None),
          ("Bz", None))


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


_REF = {}


def oracle_run(name, w, nsteps):
    if name not in _REF:
        o = orc.Oracle(w.params, **w.extras())
        st = w.state()
        dts = []
        for _ in range(nsteps):
            dt = o.compute_dt(st, w.cfl)
            o.step(st, dt)
            dts.append(dt)
        _REF[name] = (st, dts)
    return _REF[name]


CASES = {"gasrad64": lambda: wl.gasrad_box(64), "turbulence48": lambda: wl.turbulence_box(48)}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision,learned,tol", [(1, True, 1e-5), (0, False, 1e-10)])
def test_fifty_steps_against_the_oracle(mhd, name, precision, learned, tol):
    print(f"case {name} 50 steps prec={precision} learned={learned}", flush=True)
    w = CASES[name]()
    ref, dts = oracle_run(name, w, 50)
    guess = mhd.GUESS_MLP if learned else mhd.GUESS_PREV_T
    with mhd.Grid(w.params, precision=precision, eos_guess=guess) as g:
        g.load(w, mlp=eos_mlp.MLPGuess.load() if learned else None)
        for dt in dts:
            g.step(dt)
        out = g.get_state()
        diag = g.diagnostics()
    errs = {}
    for key, c in FIELDS:
        a = out[key] if c is None else out[key][c]
        b = ref[key] if c is None else ref[key][c]
        errs[f"{key}{'' if c is None else c}"] = rel_l2(a, b)
    print(name, precision, {k: f"{v:.2e}" for k, v in errs.items()}, f"divB {diag['divb_max']:.1e}",
          flush=True)
    assert all(v <= tol for v in errs.values()), errs
    assert diag["divb_max"] < 1e-12
    assert diag["fallbacks"] == 0
