"""The allocation-free CFL step, mhd_compute_dt_noalloc, against the
context's mhd_compute_dt (eq. cfl): the same kernels on the same state and
guesses give the same dt bit for bit.  Two calls in a row share the
library's device scratch, the second on a smaller grid; then a
non-physical state sets the error bits, and a clean state after it clears
them again."""
import os

import numpy as np
import pytest

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


def _dev(w):
    import torch
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t(w.U), t(w.Bx), t(w.By), t(w.Bz), t(w.T)


def _ctx_dt(mhd, w):
    with mhd.Grid(w.params) as g:
        g.load(w)
        return g.compute_dt(w.cfl)


def _noalloc_dt(mhd, w, dt_out, flags_out):
    import torch
    U, Bx, By, Bz, T = _dev(w)
    mhd.compute_dt_noalloc(w.params, U, Bx, By, Bz, T, w.cfl, dt_out, flags_out)
    torch.cuda.synchronize()
    return float(dt_out[0].item()), int(flags_out[0].item())


def test_noalloc_dt_matches_context(mhd):
    import torch
    dt_out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    flags_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    # first call: 600k cells (more than the 2048 blocks of 256 the scratch
    # holds partials for: the reduction strides), then a smaller grid
    big = wl.stratified_box(96, nz=70)
    small = wl.smooth_box(21, 13, 9, bcz=1)
    for w in (big, small):
        print(f"case noalloc dt {w.name} {w.shape}", flush=True)
        ref = _ctx_dt(mhd, w)
        got, flags = _noalloc_dt(mhd, w, dt_out, flags_out)
        assert got == ref, (w.name, got, ref)
        assert flags == 0
    # gas + radiation: the inversion from the caller's guesses, then without
    w = wl.gasrad_box(24)
    print("case noalloc dt gasrad 24^3", flush=True)
    ref = _ctx_dt(mhd, w)
    got, flags = _noalloc_dt(mhd, w, dt_out, flags_out)
    assert got == ref and flags == 0
    w.T = None
    got2, flags = _noalloc_dt(mhd, w, dt_out, flags_out)
    assert got2 == pytest.approx(ref, rel=1e-10) and flags == 0


def test_noalloc_error_bits_and_arguments(mhd):
    import torch
    dt_out = torch.zeros(1, dtype=torch.float64, device="cuda")
    flags_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    w = wl.smooth_box(12, 10, 8)
    w.U[0, 3, 4, 5] = -1.0  # negative density in one cell
    print("case noalloc non-physical cell", flush=True)
    _, flags = _noalloc_dt(mhd, w, dt_out, flags_out)
    assert flags & 1
    w = wl.smooth_box(12, 10, 8)
    _, flags = _noalloc_dt(mhd, w, dt_out, flags_out)
    assert flags == 0  # the scratch's error bits start at zero on every call
    U, Bx, By, Bz, _ = _dev(w)
    with pytest.raises(mhd.MHDError) as e:
        mhd.compute_dt_noalloc(w.params, U, Bx, By, Bz, None, -0.4, dt_out)
    assert e.value.code == -1 and "cfl" in str(e.value)
    # a grid beyond the 32-bit cell index is refused before anything runs
    # (the state pointers are never read)
    import ctypes as C
    L = mhd.load()
    d = mhd.make_desc(dict(w.params, nx=1 << 16, ny=1 << 16, nz=8))
    p = C.c_void_p(U.data_ptr())
    rc = L.mhd_compute_dt_noalloc(C.byref(d), p, p, p, p, None, 0.4,
                                  C.c_void_p(dt_out.data_ptr()), None, None)
    assert rc == -1 and b"too large" in L.mhd_last_error(None)
    # the learned guess needs a context (its weights live there)
    d = mhd.make_desc(wl.gasrad_params(8, 8, 8), eos_guess=mhd.GUESS_MLP)
    rc = L.mhd_compute_dt_noalloc(C.byref(d), p, p, p, p, None, 0.4,
                                  C.c_void_p(dt_out.data_ptr()), None, None)
    assert rc == -1 and b"previous-T" in L.mhd_last_error(None)
