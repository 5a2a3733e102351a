"""Windowed oracle evaluation for full-size parity (test helper).

One SSP-RK stage moves information by at most three cells (the two-cell
reconstruction stencil behind a face or an edge EMF, plus the face-centred
field that enters the primitives of the farthest cell), so after s stages
the interior of a sub-box with a margin of at least 3 s cells is independent
of what happens at the sub-box edges.  The oracle runs on such a window
(periodic wrap at its x/y edges, and at z edges that are not walls) and its
interior is compared with the same cells of the full-size GPU run.
"""
import collections

import numpy as np

from oracle import orc


def exact_extent(d, n):
    """A box length L with L / n == d exactly (the window keeps the cell size
    of the full grid bit for bit)."""
    L = d * n
    for _ in range(64):
        q = L / n
        if q == d:
            return L
        L = np.nextafter(L, np.inf if q < d else -np.inf)
    raise ValueError("no exact extent")


def extract(w, i0, j0, k0, nw, nzw, state=None):
    """Sub-box of nw x nw x nzw cells starting at (i0, j0, k0) (x/y wrap).
    A window whose z range touches a reflecting wall keeps that wall; its
    other z edge is treated as a wall too (far outside the compared part)."""
    p = dict(w.params)
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    st = state if state is not None else w.state(copy=False)
    ii = (i0 + np.arange(nw)) % nx
    jj = (j0 + np.arange(nw)) % ny
    reflect = p["bcz"] == 1
    if reflect:
        assert 0 <= k0 and k0 + nzw <= nz
        kk = np.arange(k0, k0 + nzw)
    else:
        kk = (k0 + np.arange(nzw)) % nz
    sel = np.ix_(kk, jj, ii)
    U = np.ascontiguousarray(st["U"][(slice(None),) + sel])
    Bx = np.ascontiguousarray(st["Bx"][sel])
    By = np.ascontiguousarray(st["By"][sel])
    if reflect:
        kf = np.arange(k0, k0 + nzw + 1)
        Bz = np.ascontiguousarray(st["Bz"][np.ix_(kf, jj, ii)])
        # walls of the window: zero normal field (exact at a real wall; at a
        # fake wall far from the compared cells it does not matter)
        Bz[0] = 0.0
        Bz[-1] = 0.0
    else:
        Bz = np.ascontiguousarray(st["Bz"][sel])
    T = None
    if st.get("T") is not None:
        T = np.ascontiguousarray(st["T"][sel])
    dx = [(p["hi"][a] - p["lo"][a]) / (nx, ny, nz)[a] for a in range(3)]
    q = dict(p, nx=nw, ny=nw, nz=nzw, lo=(0.0, 0.0, 0.0),
             hi=(exact_extent(dx[0], nw), exact_extent(dx[1], nw), exact_extent(dx[2], nzw)))
    ext = {}
    if w.bg_cc is not None:
        ext["bg_cc"] = np.ascontiguousarray(w.bg_cc[:, kk])
        ext["bg_fz"] = np.ascontiguousarray(
            w.bg_fz[:, np.arange(k0, k0 + nzw + 1)] if reflect else w.bg_fz[:, kk])
    if w.heat is not None:
        ext["heat"] = np.ascontiguousarray(w.heat[kk])
    if w.fmodes is not None:
        # the forcing of the full box, evaluated at the window's cells: the
        # window's first corner sits at (i0, j0, k0) cells from the box's
        ext["fmodes"] = w.fmodes
        ext["forcing_origin"] = (i0 * dx[0], j0 * dx[1], k0 * dx[2])
        ext["forcing_period"] = tuple(p["hi"][a] - p["lo"][a] for a in range(3))
    return q, {"U": U, "Bx": Bx, "By": By, "Bz": Bz, "T": T}, ext, (kk, jj, ii)


def oracle_window(w, dts, i0, j0, k0, nw, nzw, state=None):
    q, st, ext, idx = extract(w, i0, j0, k0, nw, nzw, state)
    o = orc.Oracle(q, **ext)
    for dt in dts:
        o.step(st, dt)
    return st, idx


Cmp = collections.namedtuple("Cmp", "dmax scale l2 l2ref n")


def compare_window(out, ref_win, idx, margin, margin_z_lo, margin_z_hi, reflect):
    """Per field over the window interior: {name: Cmp(max |gpu - oracle|,
    max |oracle|, ||gpu - oracle||_2 / ||oracle||_2, ||oracle||_2, cells)}."""
    kk, jj, ii = idx
    nzw, nw = len(kk), len(jj)
    ks = slice(margin_z_lo, nzw - margin_z_hi)
    js = slice(margin, nw - margin)
    res = {}
    for key, comps in (("U", range(5)), ("Bx", [None]), ("By", [None]), ("Bz", [None])):
        for c in comps:
            if key == "Bz" and reflect:
                sel = np.ix_(np.arange(kk[0], kk[0] + nzw + 1), jj, ii)
            else:
                sel = np.ix_(kk, jj, ii)
            g = out[key][(slice(None),) + sel][c] if c is not None else out[key][sel]
            r = ref_win[key][c] if c is not None else ref_win[key]
            diff = g[ks, js, js] - r[ks, js, js]
            rr = r[ks, js, js]
            den = float(np.sqrt(np.sum(rr * rr)))
            l2 = float(np.sqrt(np.sum(diff * diff))) / den if den > 0 else float(np.abs(diff).max())
            name = key if c is None else ("rho", "m_x", "m_y", "m_z", "E")[c]
            res[name] = Cmp(float(np.abs(diff).max()), float(np.abs(r).max()), l2, den, diff.size)
    return res
