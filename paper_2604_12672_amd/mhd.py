"""Python binding of libmhd.so (the C ABI in include/mhd.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the library.  Arrays may be numpy arrays (host) or torch CUDA
tensors (device, FP64, contiguous); the context launches on the torch
stream current at creation unless another stream is given.  The library
must have been built (``paper_2604_12672_amd.build``); importing this
module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhd.so")

HOST, DEVICE = 0, 1
PREC_FP64, PREC_SPLIT = 0, 1
GUESS_PREV_T, GUESS_MLP = 0, 1
DIFF_EINT, DIFF_TEMP = 0, 1
C_LIGHT_CODE = 2.99792458e10 / 1e8  # speed of light in units of 1e8 cm/s
RECON_VANLEER, RECON_PPH = 0, 1
BC_PERIODIC, BC_REFLECT = 0, 1

ERRORS = {-1: "MHD_ERR_ARG", -2: "MHD_ERR_NO_DEVICE", -3: "MHD_ERR_HIP",
          -4: "MHD_ERR_UNPHYSICAL", -5: "MHD_ERR_EOS", -6: "MHD_ERR_STATE"}


class MHDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("bc", C.c_int32 * 3),
        ("eos", C.c_int32), ("gamma", C.c_double), ("mu", C.c_double),
        ("rgas", C.c_double), ("arad", C.c_double), ("grav", C.c_double * 3),
        ("rk_order", C.c_int32), ("precision", C.c_int32), ("eos_guess", C.c_int32),
        ("newton_tol", C.c_double), ("newton_maxit", C.c_int32), ("mach_cut", C.c_double),
        ("xi_mode", C.c_int32), ("recon", C.c_int32), ("flatten", C.c_int32),
        ("eps_sf", C.c_double), ("nspecies", C.c_int32),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("divb_max", C.c_double), ("divb_l2", C.c_double), ("bface_max", C.c_double),
        ("total", C.c_double * 5), ("bflux_x0", C.c_double), ("newton_iters", C.c_int64),
        ("newton_max", C.c_int64), ("fallbacks", C.c_int64), ("error_flags", C.c_int32),
    ]


EXPORTS = ["mhd_init_grid", "mhd_set_background", "mhd_set_sources", "mhd_set_eos_mlp",
           "mhd_eos_solve", "mhd_set_state", "mhd_compute_dt", "mhd_step", "mhd_advance",
           "mhd_get_state", "mhd_sync", "mhd_diagnostics", "mhd_last_error", "mhd_destroy",
           "mhd_shock_flags", "mhd_set_species", "mhd_get_species",
           "mhd_launch_info", "mhd_set_opacity", "mhd_parabolic_dt", "mhd_diffuse",
           "mhd_math_check", "mhd_compute_dt_noalloc"]

_lib = None


def load():
    """Load libmhd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2604_12672_amd.build`")
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
    # the library binds to, so streams and device pointers are shared.  The
    # other order would load a second HIP runtime into the process.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.mhd_init_grid.argtypes = [C.POINTER(GridDesc), vp, C.POINTER(vp)]
    L.mhd_set_background.argtypes = [vp, vp, vp]
    L.mhd_set_sources.argtypes = [vp, vp, vp, C.c_int32]
    L.mhd_set_eos_mlp.argtypes = [vp, vp, vp, vp, vp, vp, C.c_float, vp]
    L.mhd_eos_solve.argtypes = [vp, vp, vp, vp, C.c_int64, vp, vp, C.POINTER(C.c_int64)]
    L.mhd_set_state.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32]
    L.mhd_compute_dt.argtypes = [vp, C.c_double, C.POINTER(C.c_double)]
    L.mhd_step.argtypes = [vp, C.c_double]
    L.mhd_advance.argtypes = [vp, C.c_double, C.c_int32]
    L.mhd_get_state.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32]
    L.mhd_sync.argtypes = [vp]
    L.mhd_shock_flags.argtypes = [vp, vp, C.c_int32]
    L.mhd_set_species.argtypes = [vp, vp, C.c_int32]
    L.mhd_get_species.argtypes = [vp, vp, C.c_int32]
    L.mhd_diagnostics.argtypes = [vp, C.POINTER(Diag)]
    L.mhd_last_error.argtypes = [vp]
    L.mhd_last_error.restype = C.c_char_p
    L.mhd_destroy.argtypes = [vp]
    L.mhd_math_check.argtypes = [vp, vp, C.c_int64, vp]
    L.mhd_launch_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]
    L.mhd_set_opacity.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
    L.mhd_parabolic_dt.argtypes = [vp, C.POINTER(C.c_double)]
    L.mhd_diffuse.argtypes = [vp, C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.mhd_compute_dt_noalloc.argtypes = [C.POINTER(GridDesc), vp, vp, vp, vp, vp, C.c_double,
                                         vp, vp, vp]
    for name in EXPORTS:
        getattr(L, name).restype = C.c_int if name != "mhd_last_error" else C.c_char_p
    _lib = L
    return L


def make_desc(params: dict, precision=PREC_FP64, eos_guess=GUESS_PREV_T) -> GridDesc:
    p = params
    d = GridDesc()
    d.nx, d.ny, d.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    lo, hi = p.get("lo", (0.0, 0.0, 0.0)), p.get("hi", (1.0, 1.0, 1.0))
    for a in range(3):
        d.lo[a], d.hi[a] = float(lo[a]), float(hi[a])
    d.bc[0] = d.bc[1] = BC_PERIODIC
    d.bc[2] = int(p.get("bcz", BC_PERIODIC))
    d.eos = int(p.get("eos", 0))
    d.gamma = float(p.get("gamma", 5.0 / 3.0))
    d.mu = float(p.get("mu", 0.6))
    d.rgas = float(p.get("rgas", 0.0))
    d.arad = float(p.get("arad", 0.0))
    d.grav[0], d.grav[1], d.grav[2] = 0.0, 0.0, float(p.get("gz", 0.0))
    d.rk_order = int(p.get("rk_order", 2))
    d.precision = int(precision)
    d.eos_guess = int(eos_guess)
    d.newton_tol = float(p.get("newton_tol", 1e-11))
    d.newton_maxit = int(p.get("newton_maxit", 50))
    d.mach_cut = float(p.get("mach_cut", 0.6))
    d.xi_mode = int(p.get("xi_mode", 0))
    d.recon = int(p.get("recon", RECON_VANLEER))
    d.flatten = int(p.get("flatten", 0))
    d.eps_sf = float(p.get("eps_sf", 0.2))
    d.nspecies = int(p.get("nspecies", 0))
    return d


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, where):
    """(pointer, where) of an array argument; None passes NULL."""
    if a is None:
        return None
    if _is_torch(a):
        import torch
        assert a.is_cuda and a.dtype == torch.float64 and a.is_contiguous(), \
            "device arrays must be contiguous float64 CUDA tensors"
        if where not in (None, DEVICE):
            raise ValueError("mixed host/device arguments")
        return C.c_void_p(a.data_ptr())
    a = np.asarray(a)
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "host arrays must be C-contiguous float64"
    if where not in (None, HOST):
        raise ValueError("mixed host/device arguments")
    return a.ctypes.data_as(C.c_void_p)


def _where(*arrays):
    kinds = {DEVICE if _is_torch(a) else HOST for a in arrays if a is not None}
    if len(kinds) > 1:
        raise ValueError("mixed host/device arguments")
    return kinds.pop() if kinds else HOST


def math_check(x):
    """Device reciprocal and square root of the kernels at the positive
    doubles x (a CUDA tensor): a (4, n) tensor of 1/x (EOS, primitives,
    updates), 1/x (flux arithmetic), sqrt(x) (full), sqrt(x) (flux
    arithmetic)."""
    import torch
    L = load()
    x = x.contiguous()
    out = torch.empty((4, x.numel()), dtype=torch.float64, device=x.device)
    stream = torch.cuda.current_stream(x.device).cuda_stream
    rc = L.mhd_math_check(x.data_ptr(), out.data_ptr(), x.numel(), stream)
    if rc != 0:
        raise MHDError(rc, "mhd_math_check failed")
    return out


def compute_dt_noalloc(params: dict, U, Bx, By, Bz, T, cfl, dt_out, flags_out=None,
                       stream=None):
    """CFL step of a state held in CUDA float64 tensors, without a context
    and without allocating: dt into dt_out (a one-element CUDA float64
    tensor) and the error bits into flags_out (a one-element CUDA int32
    tensor, optional), asynchronously on `stream` (default: torch's current
    stream)."""
    import torch
    L = load()
    d = make_desc(params)
    assert dt_out.is_cuda and dt_out.dtype == torch.float64 and dt_out.numel() >= 1
    if flags_out is not None:
        assert flags_out.is_cuda and flags_out.dtype == torch.int32 and flags_out.numel() >= 1
    nz, ny, nx = d.nz, d.ny, d.nx
    nzf = nz + 1 if d.bc[2] == BC_REFLECT else nz
    assert tuple(U.shape) == (5, nz, ny, nx) and tuple(Bx.shape) == (nz, ny, nx)
    assert tuple(By.shape) == (nz, ny, nx) and tuple(Bz.shape) == (nzf, ny, nx)
    if T is not None:
        assert tuple(T.shape) == (nz, ny, nx)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    rc = L.mhd_compute_dt_noalloc(C.byref(d), _ptr(U, DEVICE), _ptr(Bx, DEVICE),
                                  _ptr(By, DEVICE), _ptr(Bz, DEVICE), _ptr(T, DEVICE),
                                  float(cfl), C.c_void_p(dt_out.data_ptr()),
                                  None if flags_out is None else C.c_void_p(flags_out.data_ptr()),
                                  C.c_void_p(stream))
    if rc != 0:
        raise MHDError(rc, L.mhd_last_error(None).decode())


class Grid:
    """One library context: a grid, its device state and its stream."""

    def __init__(self, params: dict, precision=PREC_FP64, eos_guess=GUESS_PREV_T, stream=None):
        L = load()
        self._L = L
        self.params = dict(params)
        self.desc = make_desc(params, precision, eos_guess)
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
            except ImportError:
                stream = 0
        self.stream = stream
        h = C.c_void_p()
        rc = L.mhd_init_grid(C.byref(self.desc), C.c_void_p(stream), C.byref(h))
        if rc != 0:
            raise MHDError(rc, L.mhd_last_error(None).decode())
        self._h = h
        nz = self.desc.nz
        self.nzf = nz + 1 if self.desc.bc[2] == BC_REFLECT else nz
        self.shape = (nz, self.desc.ny, self.desc.nx)

    def _check(self, rc):
        if rc != 0:
            raise MHDError(rc, self._L.mhd_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.mhd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- inputs ----------------------------------------------------------
    def set_background(self, bg_cc, bg_fz):
        bg_cc = np.ascontiguousarray(bg_cc, dtype=np.float64)
        bg_fz = np.ascontiguousarray(bg_fz, dtype=np.float64)
        assert bg_cc.shape == (4, self.shape[0]) and bg_fz.shape == (4, self.nzf)
        self._check(self._L.mhd_set_background(self._h, _ptr(bg_cc, HOST), _ptr(bg_fz, HOST)))

    def set_sources(self, heat=None, fmodes=None):
        """Heating profile [nz] and forcing modes [nmodes][7] = (k_x, k_y, k_z,
        a_x, a_y, a_z, phase) (host arrays, either may be None)."""
        if heat is not None:
            heat = np.ascontiguousarray(heat, dtype=np.float64)
            assert heat.shape == (self.shape[0],)
        n = 0
        if fmodes is not None:
            fmodes = np.ascontiguousarray(fmodes, dtype=np.float64).reshape(-1, 7)
            n = len(fmodes)
        self._check(self._L.mhd_set_sources(self._h, _ptr(heat, HOST), _ptr(fmodes, HOST), n))

    def set_eos_mlp(self, model):
        """Upload a paper_2604_12672_amd.eos_mlp.MLPGuess."""
        w1, b1, w2, b2, w3, b3, norm = model.ctypes_args()
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        self._keep_mlp = (w1, b1, w2, b2, w3, norm)
        self._check(self._L.mhd_set_eos_mlp(self._h, p(w1), p(b1), p(w2), p(b2), p(w3),
                                            C.c_float(b3), p(norm)))

    def eos_solve(self, rho, e, T_guess=None, with_guess=False, stats=True, out=None):
        """Invert T(rho, e) on the device for torch CUDA float64 tensors.
        Returns (T, T0 or None, (newton steps, max steps, bracketed solves)
        or None).  stats=False makes the call asynchronous."""
        import torch
        n = rho.numel()
        T = torch.empty_like(rho) if out is None else out
        T0 = torch.empty_like(rho) if with_guess else None
        st = (C.c_int64 * 3)() if stats else None
        self._check(self._L.mhd_eos_solve(self._h, _ptr(rho, DEVICE), _ptr(e, DEVICE),
                                          _ptr(T_guess, DEVICE), n, _ptr(T, DEVICE),
                                          _ptr(T0, DEVICE), st))
        return T, T0, (tuple(st) if stats else None)

    def set_state(self, U, Bx, By, Bz, T=None):
        w = _where(U, Bx, By, Bz, T)
        self._check_shapes(U, Bx, By, Bz, T)
        self._check(self._L.mhd_set_state(self._h, _ptr(U, w), _ptr(Bx, w), _ptr(By, w),
                                          _ptr(Bz, w), _ptr(T, w), w))

    def _check_shapes(self, U, Bx, By, Bz, T):
        sh = self.shape
        assert tuple(U.shape) == (5,) + sh, U.shape
        assert tuple(Bx.shape) == sh and tuple(By.shape) == sh
        assert tuple(Bz.shape) == (self.nzf,) + sh[1:]
        if T is not None:
            assert tuple(T.shape) == sh

    def load(self, w, guess=True, mlp=None):
        """Set state, background and sources from a workloads.Workload (and
        the guess network for MHD_GUESS_MLP contexts)."""
        if mlp is not None:
            self.set_eos_mlp(mlp)
        if w.bg_cc is not None:
            self.set_background(w.bg_cc, w.bg_fz)
        if w.heat is not None or w.fmodes is not None:
            self.set_sources(w.heat, w.fmodes)
        ns = int(w.params.get("nspecies", 0))
        self.set_state(np.ascontiguousarray(w.U[:5]) if ns else w.U, w.Bx, w.By, w.Bz,
                       w.T if guess else None)
        if ns:
            self.set_species(w.U[5:])

    def set_species(self, rhoX):
        """Partial densities rho X_l [ns][nz][ny][nx] (numpy or CUDA tensor)."""
        w = _where(rhoX)
        if not _is_torch(rhoX):
            rhoX = np.ascontiguousarray(rhoX, dtype=np.float64)
        assert tuple(rhoX.shape) == (self.desc.nspecies,) + self.shape
        self._check(self._L.mhd_set_species(self._h, _ptr(rhoX, w), w))

    def get_species(self, out=None):
        if out is None:
            out = np.empty((self.desc.nspecies,) + self.shape)
        w = _where(out)
        assert tuple(out.shape) == (self.desc.nspecies,) + self.shape
        self._check(self._L.mhd_get_species(self._h, _ptr(out, w), w))
        return out

    # -- stepping --------------------------------------------------------
    def step(self, dt):
        self._check(self._L.mhd_step(self._h, float(dt)))

    def advance(self, cfl, nsteps):
        self._check(self._L.mhd_advance(self._h, float(cfl), int(nsteps)))

    def compute_dt(self, cfl):
        out = C.c_double(0.0)
        self._check(self._L.mhd_compute_dt(self._h, float(cfl), C.byref(out)))
        return out.value

    def sync(self):
        self._check(self._L.mhd_sync(self._h))

    # -- outputs ---------------------------------------------------------
    def get_state(self, out=None, with_T=False):
        """Return the state as numpy arrays, or copy into `out` (a dict of
        arrays or tensors with the keys U, Bx, By, Bz[, T])."""
        if out is None:
            sh = self.shape
            out = {"U": np.empty((5,) + sh), "Bx": np.empty(sh), "By": np.empty(sh),
                   "Bz": np.empty((self.nzf,) + sh[1:])}
            if with_T:
                out["T"] = np.empty(sh)
        T = out.get("T")
        w = _where(out["U"], out["Bx"], out["By"], out["Bz"], T)
        self._check_shapes(out["U"], out["Bx"], out["By"], out["Bz"], T)
        self._check(self._L.mhd_get_state(self._h, _ptr(out["U"], w), _ptr(out["Bx"], w),
                                          _ptr(out["By"], w), _ptr(out["Bz"], w), _ptr(T, w), w))
        return out

    def shock_flags(self, out=None):
        """Shock-flattening flags of the current state (uint8 per cell), into
        `out` (a uint8 numpy array or CUDA tensor of the grid's shape) or a
        new numpy array."""
        if out is None:
            out = np.empty(self.shape, dtype=np.uint8)
        if _is_torch(out):
            import torch
            assert out.is_cuda and out.dtype == torch.uint8 and out.is_contiguous()
            assert tuple(out.shape) == self.shape
            ptr, w = C.c_void_p(out.data_ptr()), DEVICE
        else:
            assert out.dtype == np.uint8 and out.flags["C_CONTIGUOUS"] and out.shape == self.shape
            ptr, w = out.ctypes.data_as(C.c_void_p), HOST
        self._check(self._L.mhd_shock_flags(self._h, ptr, w))
        return out

    def diagnostics(self):
        d = Diag()
        self._check(self._L.mhd_diagnostics(self._h, C.byref(d)))
        return {"divb_max": d.divb_max, "divb_l2": d.divb_l2, "bface_max": d.bface_max,
                "total": list(d.total), "bflux_x0": d.bflux_x0,
                "newton_iters": d.newton_iters, "newton_max": d.newton_max,
                "fallbacks": d.fallbacks, "error_flags": d.error_flags}

    # -- thermal diffusion (RKL2) --------------------------------------------
    def set_opacity(self, kappa0, alpha=0.0, beta=0.0, clight=C_LIGHT_CODE):
        self._check(self._L.mhd_set_opacity(self._h, float(kappa0), float(alpha), float(beta),
                                            float(clight)))

    def parabolic_dt(self):
        out = C.c_double(0.0)
        self._check(self._L.mhd_parabolic_dt(self._h, C.byref(out)))
        return out.value

    def diffuse(self, dt, nsts=0, mode=DIFF_EINT):
        """One RKL2 step; returns the number of stages used."""
        used = C.c_int32(0)
        self._check(self._L.mhd_diffuse(self._h, float(dt), int(nsts), int(mode), C.byref(used)))
        return used.value

    def launch_info(self):
        t, z, b = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self._L.mhd_launch_info(self._h, C.byref(t), C.byref(z), C.byref(b)))
        return {"tile": t.value, "zseg": z.value, "blocks": b.value}
