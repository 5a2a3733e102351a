"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this module.  It marshals numpy arrays into the C oracle and adds no
arithmetic of its own.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmhd_oracle.so")
_lib = None

BC_PERIODIC, BC_REFLECT = 0, 1
EOS_IDEAL, EOS_GASRAD = 0, 1
XI_LINEAR, XI_STEP, XI_OFF = 0, 1, 2
RECON_VANLEER, RECON_PPH = 0, 1

_DP = C.POINTER(C.c_double)


class _Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("bcz", C.c_int), ("eos", C.c_int),
        ("gamma", C.c_double), ("mu", C.c_double), ("rgas", C.c_double),
        ("arad", C.c_double), ("gz", C.c_double),
        ("rk_order", C.c_int), ("newton_tol", C.c_double),
        ("newton_maxit", C.c_int), ("mach_cut", C.c_double),
        ("xi_mode", C.c_int), ("recon", C.c_int),
        ("flatten", C.c_int), ("eps_sf", C.c_double), ("nspecies", C.c_int),
        ("bg_cc", _DP), ("bg_fz", _DP), ("heat", _DP), ("force", _DP),
    ]


class _Opacity(C.Structure):
    _fields_ = [("kappa0", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("clight", C.c_double)]


DIFF_EINT, DIFF_TEMP = 0, 1
C_LIGHT_CODE = 2.99792458e10 / 1e8  # speed of light in units of 1e8 cm/s


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # noqa: F401  (package import)
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        L = _lib
        L.orc_step.argtypes = [C.POINTER(_Cfg), _DP, _DP, _DP, _DP, _DP, C.c_double]
        L.orc_residual.argtypes = [C.POINTER(_Cfg)] + [_DP] * 10
        L.orc_compute_dt.argtypes = [C.POINTER(_Cfg), _DP, _DP, _DP, _DP, _DP,
                                     C.c_double, _DP]
        L.orc_forcing.argtypes = [C.POINTER(_Cfg), _DP, C.c_int, _DP, _DP, _DP]
        L.orc_forcing.restype = None
        L.orc_divb.argtypes = [C.POINTER(_Cfg), _DP, _DP, _DP, _DP]
        L.orc_divb.restype = None
        L.orc_primitives.argtypes = [C.POINTER(_Cfg)] + [_DP] * 7
        L.orc_riemann.argtypes = [C.POINTER(_Cfg), _DP, _DP, C.c_double, _DP]
        L.orc_hll.argtypes = [C.POINTER(_Cfg), _DP, _DP, C.c_double, _DP]
        L.orc_shock_flags.argtypes = [C.POINTER(_Cfg)] + [_DP] * 5 + [C.POINTER(C.c_ubyte)]
        L.orc_eos_invert.argtypes = [C.POINTER(_Cfg), C.c_double, C.c_double,
                                     C.c_double, _DP, C.POINTER(C.c_int),
                                     C.POINTER(C.c_int)]
        L.orc_eos_thermo.argtypes = [C.POINTER(_Cfg), C.c_double, C.c_double,
                                     _DP, _DP, _DP, _DP]
        L.orc_vanleer.argtypes = [C.c_double, C.c_double]
        L.orc_pph.argtypes = [C.c_double, C.c_double, C.c_double, _DP, _DP]
        L.orc_pph.restype = None
        L.orc_pph_limited.argtypes = [C.c_double, C.c_double, C.c_double, _DP, _DP]
        L.orc_pph_limited.restype = None
        OP = C.POINTER(_Opacity)
        L.orc_diffusion_rhs.argtypes = [C.POINTER(_Cfg), OP, _DP, _DP, _DP]
        L.orc_parabolic_dt.argtypes = [C.POINTER(_Cfg), OP, _DP, _DP, _DP]
        L.orc_rkl2_nsts.argtypes = [C.c_double, C.c_double]
        L.orc_rkl2_coeffs.argtypes = [C.c_int, C.c_int, _DP, _DP, _DP, _DP]
        L.orc_rkl2_coeffs.restype = None
        L.orc_diffuse.argtypes = [C.POINTER(_Cfg), OP, _DP, _DP, _DP, _DP, _DP, C.c_double,
                                  C.c_int, C.c_int]
        L.orc_vanleer.restype = C.c_double
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "need C-contiguous float64"
    return a.ctypes.data_as(_DP)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


DEFAULTS = dict(
    bcz=BC_PERIODIC, eos=EOS_IDEAL, gamma=5.0 / 3.0, mu=0.6, rgas=0.0, arad=0.0,
    gz=0.0, rk_order=2, newton_tol=1e-11, newton_maxit=50, mach_cut=0.6,
    xi_mode=XI_LINEAR, recon=RECON_VANLEER, flatten=0, eps_sf=0.2, nspecies=0,
)


class Oracle:
    """The oracle bound to one problem description (a dict of grid and
    physics parameters, plus optional background and heating arrays, and a
    forcing given as an acceleration field or as Fourier modes).

    fmodes [nmodes][7] = (k_x, k_y, k_z, a_x, a_y, a_z, phi): the forcing
    sum_m a_m cos(2 pi k_m . (x / L) + phi_m), evaluated at the cell centres
    by orc_forcing; x is measured from the forcing's reference corner, which
    lies at -forcing_origin from this grid's first cell corner (a window of a
    larger grid passes its offset), L = forcing_period (default: this box)."""

    def __init__(self, params: dict, bg_cc=None, bg_fz=None, heat=None, force=None,
                 fmodes=None, forcing_origin=(0.0, 0.0, 0.0), forcing_period=None):
        p = dict(DEFAULTS)
        p.update(params)
        self.p = p
        nx, ny, nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
        lo, hi = p.get("lo", (0.0, 0.0, 0.0)), p.get("hi", (1.0, 1.0, 1.0))
        self.shape = (nz, ny, nx)
        self.nzf = nz + 1 if p["bcz"] == BC_REFLECT else nz
        if fmodes is not None:
            assert force is None, "give the forcing as a field or as modes, not both"
            period = forcing_period or tuple(hi[a] - lo[a] for a in range(3))
            force = self.forcing_field(fmodes, forcing_origin, period)
        self._keep = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                      for a in (bg_cc, bg_fz, heat, force)]
        bcc, bfz, ht, fc = self._keep
        self.cfg = _Cfg(
            nx, ny, nz,
            (hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / ny, (hi[2] - lo[2]) / nz,
            int(p["bcz"]), int(p["eos"]), float(p["gamma"]), float(p["mu"]),
            float(p["rgas"]), float(p["arad"]), float(p["gz"]), int(p["rk_order"]),
            float(p["newton_tol"]), int(p["newton_maxit"]), float(p["mach_cut"]),
            int(p["xi_mode"]), int(p["recon"]), int(p["flatten"]), float(p["eps_sf"]),
            int(p["nspecies"]), _ptr(bcc), _ptr(bfz), _ptr(ht), _ptr(fc),
        )

    def forcing_field(self, fmodes, origin, period):
        """[3][nz][ny][nx] acceleration of the Fourier modes (orc_forcing)."""
        nx, ny, nz = int(self.p["nx"]), int(self.p["ny"]), int(self.p["nz"])
        lo, hi = self.p.get("lo", (0.0, 0.0, 0.0)), self.p.get("hi", (1.0, 1.0, 1.0))
        cfg = _Cfg(nx, ny, nz, (hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / ny,
                   (hi[2] - lo[2]) / nz)
        m = np.ascontiguousarray(fmodes, dtype=np.float64).reshape(-1, 7)
        o = np.ascontiguousarray(origin, dtype=np.float64)
        L = np.ascontiguousarray(period, dtype=np.float64)
        out = np.empty((3, nz, ny, nx))
        lib().orc_forcing(C.byref(cfg), _ptr(m), len(m), _ptr(o), _ptr(L), _ptr(out))
        return out

    # -- state helpers -------------------------------------------------
    def _state(self, st):
        U = st["U"]
        for k in ("U", "Bx", "By", "Bz"):
            assert st[k].dtype == np.float64 and st[k].flags["C_CONTIGUOUS"], k
        assert U.shape == (5 + int(self.p["nspecies"]),) + self.shape
        T = st.get("T")
        if self.p["eos"] == EOS_GASRAD:
            assert T is not None and T.shape == self.shape
        return U, st["Bx"], st["By"], st["Bz"], T

    def step(self, st: dict, dt: float) -> None:
        U, Bx, By, Bz, T = self._state(st)
        _check(lib().orc_step(C.byref(self.cfg), _ptr(U), _ptr(Bx), _ptr(By), _ptr(Bz),
                              _ptr(T), float(dt)), "orc_step")

    def residual(self, st: dict):
        U, Bx, By, Bz, T = self._state(st)
        RU = np.empty_like(U)
        RBx, RBy, RBz = np.empty_like(Bx), np.empty_like(By), np.empty_like(Bz)
        Tout = None if T is None else np.empty_like(T)
        _check(lib().orc_residual(C.byref(self.cfg), _ptr(U), _ptr(Bx), _ptr(By), _ptr(Bz),
                                  _ptr(T), _ptr(Tout), _ptr(RU), _ptr(RBx), _ptr(RBy),
                                  _ptr(RBz)), "orc_residual")
        return RU, RBx, RBy, RBz, Tout

    # -- thermal diffusion (Sect. 2.10) ----------------------------------
    def diffuse(self, st: dict, dt: float, nsts: int, op, mode=DIFF_EINT) -> None:
        """One RKL2 step of thermal diffusion; updates st["U"][4] and st["T"]."""
        U, Bx, By, Bz, T = self._state(st)
        _check(lib().orc_diffuse(C.byref(self.cfg), C.byref(op), _ptr(U), _ptr(Bx), _ptr(By),
                                 _ptr(Bz), _ptr(T), float(dt), int(nsts), int(mode)),
               "orc_diffuse")

    def diffusion_rhs(self, rho, T, op):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        M = np.empty_like(T)
        _check(lib().orc_diffusion_rhs(C.byref(self.cfg), C.byref(op), _ptr(rho), _ptr(T),
                                       _ptr(M)), "orc_diffusion_rhs")
        return M

    def parabolic_dt(self, rho, T, op) -> float:
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        out = C.c_double(0.0)
        _check(lib().orc_parabolic_dt(C.byref(self.cfg), C.byref(op), _ptr(rho), _ptr(T),
                                      C.byref(out)), "orc_parabolic_dt")
        return out.value

    def compute_dt(self, st: dict, cfl: float) -> float:
        U, Bx, By, Bz, T = self._state(st)
        out = C.c_double(0.0)
        _check(lib().orc_compute_dt(C.byref(self.cfg), _ptr(U), _ptr(Bx), _ptr(By),
                                    _ptr(Bz), _ptr(T), float(cfl), C.byref(out)),
               "orc_compute_dt")
        return out.value

    def divb(self, st: dict):
        out = np.empty(self.shape)
        lib().orc_divb(C.byref(self.cfg), _ptr(st["Bx"]), _ptr(st["By"]), _ptr(st["Bz"]),
                       _ptr(out))
        return out

    def primitives(self, st: dict):
        U, Bx, By, Bz, T = self._state(st)
        out = np.empty((10,) + self.shape)
        Tout = None if T is None else np.empty_like(T)
        _check(lib().orc_primitives(C.byref(self.cfg), _ptr(U), _ptr(Bx), _ptr(By),
                                    _ptr(Bz), _ptr(T), _ptr(Tout), _ptr(out)),
               "orc_primitives")
        return out, Tout

    # -- pointwise routines -------------------------------------------
    def riemann(self, WL, WR, bn):
        WL = np.ascontiguousarray(WL, dtype=np.float64)
        WR = np.ascontiguousarray(WR, dtype=np.float64)
        F = np.empty(7)
        _check(lib().orc_riemann(C.byref(self.cfg), _ptr(WL), _ptr(WR), float(bn), _ptr(F)),
               "orc_riemann")
        return F

    def hll(self, WL, WR, bn):
        WL = np.ascontiguousarray(WL, dtype=np.float64)
        WR = np.ascontiguousarray(WR, dtype=np.float64)
        F = np.empty(7)
        _check(lib().orc_hll(C.byref(self.cfg), _ptr(WL), _ptr(WR), float(bn), _ptr(F)),
               "orc_hll")
        return F

    def shock_flags(self, st: dict) -> np.ndarray:
        """Shock-flattening flags (0/1, uint8) of every cell of the state."""
        U, Bx, By, Bz, T = self._state(st)
        out = np.zeros(self.shape, dtype=np.uint8)
        _check(lib().orc_shock_flags(C.byref(self.cfg), _ptr(U), _ptr(Bx), _ptr(By), _ptr(Bz),
                                     _ptr(T), out.ctypes.data_as(C.POINTER(C.c_ubyte))),
               "orc_shock_flags")
        return out

    def eos_invert(self, rho, eint, tguess):
        T = C.c_double(0.0)
        it, fb = C.c_int(0), C.c_int(0)
        _check(lib().orc_eos_invert(C.byref(self.cfg), float(rho), float(eint), float(tguess),
                                    C.byref(T), C.byref(it), C.byref(fb)), "orc_eos_invert")
        return T.value, it.value, fb.value

    def eos_thermo(self, rho, T):
        P, e, cv, cs2 = (C.c_double(0.0) for _ in range(4))
        lib().orc_eos_thermo(C.byref(self.cfg), float(rho), float(T), C.byref(P), C.byref(e),
                             C.byref(cv), C.byref(cs2))
        return P.value, e.value, cv.value, cs2.value


def opacity(kappa0, alpha=0.0, beta=0.0, clight=C_LIGHT_CODE):
    """Opacity law kappa = kappa0 rho^alpha T^beta (thermal diffusion)."""
    return _Opacity(float(kappa0), float(alpha), float(beta), float(clight))


def rkl2_nsts(dt_h: float, dt_p: float) -> int:
    return lib().orc_rkl2_nsts(float(dt_h), float(dt_p))


def rkl2_coeffs(s: int, j: int):
    """(mu, nu, mu~, gamma~) of stage j of an s-stage RKL2 step."""
    v = [C.c_double() for _ in range(4)]
    lib().orc_rkl2_coeffs(int(s), int(j), *[C.byref(x) for x in v])
    return tuple(x.value for x in v)


def vanleer(a: float, b: float) -> float:
    return lib().orc_vanleer(float(a), float(b))


def pph(wm: float, wc: float, wp: float):
    """(lower, upper) face values of the PPH parabola of a cell."""
    lo, hi = C.c_double(), C.c_double()
    lib().orc_pph(float(wm), float(wc), float(wp), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def pph_limited(wm: float, wc: float, wp: float):
    """(lower, upper) face values of the limited parabola of a mass fraction."""
    lo, hi = C.c_double(), C.c_double()
    lib().orc_pph_limited(float(wm), float(wc), float(wp), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return lib().orc_num_threads()
