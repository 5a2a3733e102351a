"""The windowed oracle evaluation used for full-size parity reproduces the
oracle's full-grid step exactly inside the margin (CPU)."""
import os
import sys

import numpy as np
import pytest

from oracle import orc
from paper_2604_12672_amd import workloads as wl

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import window  # noqa: E402


@pytest.mark.parametrize("case", ["stratified_wall", "stratified_interior", "gasrad_periodic"])
def test_window_matches_full_grid(case):
    if case.startswith("stratified"):
        w = wl.stratified_box(36, nz=48, heating=True)
    else:
        w = wl.smooth_box(36, 36, 36, eos=wl.EOS_GASRAD)
    o = orc.Oracle(w.params, **w.extras())
    full = w.state()
    dts = []
    for _ in range(2):
        dt = o.compute_dt(full, 0.4)
        o.step(full, dt)
        dts.append(dt)
    # two SSP-RK2 steps = four stages of three cells each
    margin = 12
    if case == "stratified_wall":
        k0, nzw, mlo, mhi = 0, 30, 0, margin
    elif case == "stratified_interior":
        k0, nzw, mlo, mhi = 9, 30, margin, margin
    else:
        k0, nzw, mlo, mhi = 25, 30, margin, margin  # wraps in periodic z
    win, idx = window.oracle_window(w, dts, 27, 5, k0, 30, nzw)
    res = window.compare_window(full, win, idx, margin, mlo, mhi, w.params["bcz"] == 1)
    for name, c in res.items():
        assert c.dmax == 0.0, (case, name, c)
