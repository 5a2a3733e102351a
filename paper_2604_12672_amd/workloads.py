"""Seeded synthetic inputs for the MHD step (initial states, backgrounds,
source profiles).

This module builds input arrays only: it holds none of the scheme's
arithmetic (no reconstruction, Riemann solver, EMFs or EOS inversion), and
both the HIP library and the FP64 oracle consume what it produces.  Every
random draw comes from ``numpy.random.default_rng(seed)``.

Array layout (FP64, x fastest): U[5][nz][ny][nx] = (rho, m_x, m_y, m_z, E);
Bx[nz][ny][nx], By[nz][ny][nx] hold the lower x/y faces of each cell;
Bz[nzf][ny][nx] the lower z faces (nzf = nz+1 with reflecting z walls).
E = rho e_int + rho |v|^2 / 2 + |B_cc|^2 / 2 with B_cc the face mean.

Units: the gas+radiation workloads use rho in g/cm^3, velocities in
1e8 cm/s and T in kelvin, so the gas constant and the radiation constant
become R = k_B/(m_u (1e8 cm/s)^2) and a = a_rad/(1 g cm^-3 (1e8 cm/s)^2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BC_PERIODIC, BC_REFLECT = 0, 1
EOS_IDEAL, EOS_GASRAD = 0, 1

K_B = 1.380649e-16          # erg/K
M_U = 1.66053906660e-24     # g
A_RAD = 7.565723e-15        # erg cm^-3 K^-4
V_UNIT = 1.0e8              # cm/s
R_CODE = K_B / (M_U * V_UNIT ** 2)
A_CODE = A_RAD / (V_UNIT ** 2)


@dataclasses.dataclass
class Workload:
    name: str
    params: dict
    U: np.ndarray
    Bx: np.ndarray
    By: np.ndarray
    Bz: np.ndarray
    T: np.ndarray | None = None
    bg_cc: np.ndarray | None = None   # [4][nz] rho, P, gamma_e, gamma_c
    bg_fz: np.ndarray | None = None   # [4][nzf]
    heat: np.ndarray | None = None    # [nz]
    fmodes: np.ndarray | None = None  # [nmodes][7] forcing (k, a, phase)
    cfl: float = 0.4
    steps: int = 1

    @property
    def shape(self):
        p = self.params
        return (p["nz"], p["ny"], p["nx"])

    @property
    def ncells(self):
        p = self.params
        return p["nx"] * p["ny"] * p["nz"]

    def state(self, copy=True):
        f = (lambda a: None if a is None else a.copy()) if copy else (lambda a: a)
        return {"U": f(self.U), "Bx": f(self.Bx), "By": f(self.By), "Bz": f(self.Bz),
                "T": f(self.T)}

    def extras(self):
        return dict(bg_cc=self.bg_cc, bg_fz=self.bg_fz, heat=self.heat, fmodes=self.fmodes)


def base_params(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), **kw):
    p = dict(nx=int(nx), ny=int(ny), nz=int(nz), lo=tuple(map(float, lo)),
             hi=tuple(map(float, hi)), bcz=BC_PERIODIC, eos=EOS_IDEAL, gamma=5.0 / 3.0,
             mu=0.6, rgas=0.0, arad=0.0, gz=0.0, rk_order=2, newton_tol=1e-11,
             newton_maxit=50, mach_cut=0.6, xi_mode=0)
    p.update(kw)
    return p


def _centres(p):
    lo, hi = p["lo"], p["hi"]
    n = (p["nx"], p["ny"], p["nz"])
    d = [(hi[a] - lo[a]) / n[a] for a in range(3)]
    xc = lo[0] + (np.arange(n[0]) + 0.5) * d[0]
    yc = lo[1] + (np.arange(n[1]) + 0.5) * d[1]
    zc = lo[2] + (np.arange(n[2]) + 0.5) * d[2]
    xf = lo[0] + np.arange(n[0]) * d[0]
    yf = lo[1] + np.arange(n[1]) * d[1]
    nzf = n[2] + 1 if p["bcz"] == BC_REFLECT else n[2]
    zf = lo[2] + np.arange(nzf) * d[2]
    return xc, yc, zc, xf, yf, zf, d


def _cell_field(p, Bx, By, Bz):
    bx = 0.5 * (Bx + np.roll(Bx, -1, axis=2))
    by = 0.5 * (By + np.roll(By, -1, axis=1))
    if p["bcz"] == BC_REFLECT:
        bz = 0.5 * (Bz[:-1] + Bz[1:])
    else:
        bz = 0.5 * (Bz + np.roll(Bz, -1, axis=0))
    return bx, by, bz


def _conserved(p, rho, vx, vy, vz, P, Bx, By, Bz, eint=None):
    """U from primitive point values; e_int = P/((gamma-1) rho) unless given."""
    bx, by, bz = _cell_field(p, Bx, By, Bz)
    if eint is None:
        eint = P / ((p["gamma"] - 1.0) * rho)
    U = np.empty((5,) + rho.shape)
    U[0] = rho
    U[1] = rho * vx
    U[2] = rho * vy
    U[3] = rho * vz
    U[4] = rho * eint + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (bx * bx + by * by + bz * bz)
    return U


def _curl_2d(p, Az):
    """Face field of B = curl(Az z_hat) from Az at the (x_{i-1/2}, y_{j-1/2})
    corners: Bx = dAz/dy, By = -dAz/dx (differences of corner values)."""
    _, _, _, _, _, _, d = _centres(p)
    Bx = (np.roll(Az, -1, axis=-2) - Az) / d[1]
    By = -(np.roll(Az, -1, axis=-1) - Az) / d[0]
    return Bx, By


def _full(shape, v):
    return np.full(shape, float(v))


# --------------------------------------------------------------------------
# 2D ideal-MHD tests
# --------------------------------------------------------------------------

def orszag_tang(n=64, steps=200, cfl=0.4):
    """Orszag-Tang vortex on [0,1]^2: rho = 25/(36 pi), P = 5/(12 pi),
    v = (-sin 2 pi y, sin 2 pi x), Az = B0 (cos 4 pi x/(4 pi) + cos 2 pi y/(2 pi)),
    B0 = 1/sqrt(4 pi), gamma = 5/3."""
    p = base_params(n, n, 1)
    xc, yc, _, xf, yf, _, _ = _centres(p)
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    XF, YF = np.meshgrid(xf, yf, indexing="xy")
    B0 = 1.0 / math.sqrt(4.0 * math.pi)
    Az = B0 * (np.cos(4 * np.pi * XF) / (4 * np.pi) + np.cos(2 * np.pi * YF) / (2 * np.pi))
    Bx, By = _curl_2d(p, Az)
    Bx, By = Bx[None], By[None]
    Bz = np.zeros((1, n, n))
    rho = _full((1, n, n), 25.0 / (36.0 * math.pi))
    P = _full((1, n, n), 5.0 / (12.0 * math.pi))
    vx = -np.sin(2 * np.pi * Y)[None]
    vy = np.sin(2 * np.pi * X)[None]
    U = _conserved(p, rho, vx, vy, np.zeros_like(vx), P, Bx, By, Bz)
    return Workload("orszag_tang", p, U, Bx, By, Bz, cfl=cfl, steps=steps)


def linear_wave(n=32, kind="alfven", amp=1e-6, cfl=0.4):
    """Linear wave along the grid diagonal on [0,1]^2, k = 2 pi (1,1):
    rho0 = 1, P0 = 3/5 (c_s = 1 for gamma = 5/3).
    alfven: B0 = 1 along k_hat, dv = amp sin(k.x) e_perp, dB = -sqrt(rho0) dv,
            dB set through Az = -amp cos(k.x)/|k| ... (scaled by sqrt(rho0));
    sound:  B0 = 0, drho = amp rho0 sin(k.x), dv = amp c_s sin(k.x) k_hat,
            dP = c_s^2 drho.
    The exact solution translates along k_hat at v_A (resp. c_s); one period
    is 1/sqrt(2)."""
    p = base_params(n, n, 1)
    xc, yc, _, xf, yf, _, d = _centres(p)
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    rho0, P0, gam = 1.0, 0.6, p["gamma"]
    cs = math.sqrt(gam * P0 / rho0)
    kk = 2 * math.pi * math.sqrt(2.0)
    phase = 2 * np.pi * (X + Y)
    zero = np.zeros((1, n, n))
    if kind == "alfven":
        B0 = 1.0
        # corners (x_{i-1/2}, y_{j-1/2})
        XF, YF = np.meshgrid(xf, yf, indexing="xy")
        psi = -amp * math.sqrt(rho0) * np.cos(2 * np.pi * (XF + YF)) / kk
        dBx, dBy = _curl_2d(p, psi)
        Bx = (B0 / math.sqrt(2.0) + dBx)[None]
        By = (B0 / math.sqrt(2.0) + dBy)[None]
        dv = amp * np.sin(phase)
        vx = (-dv / math.sqrt(2.0))[None]
        vy = (dv / math.sqrt(2.0))[None]
        rho = _full((1, n, n), rho0)
        P = _full((1, n, n), P0)
        speed = B0 / math.sqrt(rho0)
    elif kind == "sound":
        Bx = zero.copy()
        By = zero.copy()
        s = amp * np.sin(phase)
        rho = (rho0 * (1.0 + s))[None]
        vx = (cs * s / math.sqrt(2.0))[None]
        vy = (cs * s / math.sqrt(2.0))[None]
        P = (P0 + cs * cs * rho0 * s)[None]
        speed = cs
    else:
        raise ValueError(kind)
    Bz = zero.copy()
    U = _conserved(p, rho, vx, vy, zero, P, Bx, By, Bz)
    w = Workload(f"{kind}_wave", p, U, Bx, By, Bz, cfl=cfl)
    w.period = 1.0 / (math.sqrt(2.0) * speed)
    return w


def brio_wu(n=500, axis=0, cfl=0.4):
    """Brio-Wu shock tube: (rho, v_n, v_t, B_t, P) = (1, 0, 0, 1, 1) on the
    left, (0.125, 0, 0, -1, 0.1) on the right, B_n = 0.75, gamma = 2.  Laid
    out periodically on a line of length 2 with the left state in [0.5, 1.5),
    so the tube's two jumps are mirror images that do not interact before
    t = 0.08.  axis selects the direction of the line (0, 1 or 2); the
    transverse field is the next axis in cyclic order."""
    shape_n = [1, 1, 1]
    shape_n[axis] = n
    hi = [1.0, 1.0, 1.0]
    hi[axis] = 2.0
    p = base_params(shape_n[0], shape_n[1], shape_n[2], hi=tuple(hi), gamma=2.0)
    xc, yc, zc, *_ = _centres(p)
    s = (xc, yc, zc)[axis]
    left = (s >= 0.5) & (s < 1.5)
    shp = (p["nz"], p["ny"], p["nx"])

    def line(vl, vr):
        v = np.where(left, vl, vr)
        return np.broadcast_to(v.reshape(_line_shape(axis, n)), shp).copy()

    rho = line(1.0, 0.125)
    P = line(1.0, 0.1)
    bt = line(1.0, -1.0)
    B = [None, None, None]
    B[axis] = np.full(shp, 0.75)
    B[(axis + 1) % 3] = bt
    B[(axis + 2) % 3] = np.zeros(shp)
    zero = np.zeros(shp)
    U = _conserved(p, rho, zero, zero, zero, P, B[0], B[1], B[2])
    return Workload("brio_wu", p, U, B[0], B[1], B[2], cfl=cfl)


def _line_shape(axis, n):
    s = [1, 1, 1]  # (nz, ny, nx)
    s[2 - axis] = n
    return tuple(s)


def balsara_vortex(n=64, utilde=1e-2, beta_k=1.0, cfl=0.4):
    """Balsara (2004) vortex on (-5,5)^2 advected along the diagonal at
    u_adv = utilde (Sect. 3.2 of the paper): v, B ~ exp((1-r^2)/2)(-y, x),
    P = 1 + [B~^2 (1-r^2)/2 - u~^2/2] exp(1-r^2), rho = 1, B~ = u~ sqrt(beta_K).
    Face B comes from Az = B~ exp((1-r^2)/2) at the cell corners."""
    p = base_params(n, n, 1, lo=(-5.0, -5.0, 0.0), hi=(5.0, 5.0, 1.0))
    xc, yc, _, xf, yf, _, _ = _centres(p)
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    XF, YF = np.meshgrid(xf, yf, indexing="xy")
    bt = utilde * math.sqrt(beta_k)
    r2 = X * X + Y * Y
    ex = np.exp(0.5 * (1.0 - r2))
    vx = (utilde * ex * (-Y) + utilde / math.sqrt(2.0))[None]
    vy = (utilde * ex * X + utilde / math.sqrt(2.0))[None]
    P = (1.0 + (0.5 * bt * bt * (1.0 - r2) - 0.5 * utilde * utilde) * np.exp(1.0 - r2))[None]
    rho = np.ones((1, n, n))
    Az = bt * np.exp(0.5 * (1.0 - (XF * XF + YF * YF)))
    Bx, By = _curl_2d(p, Az)
    Bx, By = Bx[None], By[None]
    Bz = np.zeros((1, n, n))
    U = _conserved(p, rho, vx, vy, np.zeros_like(vx), P, Bx, By, Bz)
    w = Workload("balsara_vortex", p, U, Bx, By, Bz, cfl=cfl)
    w.tau = 10.0 * math.sqrt(2.0) / utilde
    return w


# --------------------------------------------------------------------------
# 3D stratified box (polytrope under constant gravity)
# --------------------------------------------------------------------------

POLY_THETA_TOP = math.exp(-1.6)   # P ~ theta^2.5: ln(P_b/P_t) = 4


def polytrope_profile(z, lz=1.0, rho_b=1.0, p_b=1.0):
    """n = 1.5 polytrope with theta = P/rho falling linearly with height from
    theta_b at z = 0 to theta_b exp(-1.6) at z = lz (four pressure scale
    heights, ln(P_b/P_t) = 4).  Returns rho, P and the gravity g_z (< 0) that
    puts it in hydrostatic equilibrium."""
    th_b = p_b / rho_b
    th = th_b * (1.0 - (1.0 - POLY_THETA_TOP) * z / lz)
    rho = rho_b * (th / th_b) ** 1.5
    P = p_b * (th / th_b) ** 2.5
    g = 2.5 * th_b * (1.0 - POLY_THETA_TOP) / lz
    return rho, P, -g


def stratified_box(n=256, nz=None, seed_rho=1, seed_b=2, beta=1e6, drho=1e-4,
                   heating=False, perturb=True, seed_field=True, steps=100, cfl=0.4):
    """Plane-parallel n = 1.5 polytrope (gamma = 5/3) on [0,1]^3, periodic in x
    and y, reflecting in z, under constant gravity.  Seeded isobaric density
    noise delta rho/rho iid uniform in [-drho, drho] (seed_rho); a weak
    solenoidal seed field with <2P>/<B^2> = beta from a random edge vector
    potential (seed_b) whose x and y components vanish on the walls.
    heating: energy source +q in z < 0.1 and -q in z > 0.9 with
    q = 1e-6 rho_b c_b^3 / 0.1.  The background (rho_hat, P_hat, gamma,
    gamma) is the exact profile at cell centres and z faces."""
    nz = n if nz is None else nz
    p = base_params(n, n, nz, bcz=BC_REFLECT)
    xc, yc, zc, xf, yf, zf, d = _centres(p)
    rho_c, P_c, g = polytrope_profile(zc)
    rho_f, P_f, _ = polytrope_profile(zf)
    p["gz"] = g
    gam = p["gamma"]
    bg_cc = np.stack([rho_c, P_c, np.full(nz, gam), np.full(nz, gam)])
    bg_fz = np.stack([rho_f, P_f, np.full(nz + 1, gam), np.full(nz + 1, gam)])
    shp = (nz, n, n)
    rho = np.broadcast_to(rho_c[:, None, None], shp).copy()
    P = np.broadcast_to(P_c[:, None, None], shp).copy()
    if perturb:
        rng = np.random.default_rng(seed_rho)
        rho *= 1.0 + rng.uniform(-drho, drho, size=shp)
    Bx = np.zeros(shp)
    By = np.zeros(shp)
    Bz = np.zeros((nz + 1, n, n))
    if seed_field:
        Bx, By, Bz = _seed_field(p, seed_b, P, beta)
    zero = np.zeros(shp)
    U = _conserved(p, rho, zero, zero, zero, P, Bx, By, Bz)
    heat = None
    if heating:
        cb = math.sqrt(gam * 1.0 / 1.0)
        q = 1e-6 * 1.0 * cb ** 3 / 0.1
        heat = np.where(zc < 0.1, q, np.where(zc > 0.9, -q, 0.0))
    w = Workload("stratified_box", p, U, Bx, By, Bz, bg_cc=bg_cc, bg_fz=bg_fz, heat=heat,
                 cfl=cfl, steps=steps)
    return w


def _seed_field(p, seed, P, beta, kmax=4, nmodes=12):
    """Random solenoidal face field from an edge vector potential
    A = (A_x, A_y, 0) with A_x, A_y = sum of modes
    a cos(2 pi (kx x + ky y) + phi) sin(m pi z), 1 <= |k_perp| <= kmax,
    m in {1, 2}; zero on the z walls, so B_z = 0 there."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    xc, yc, zc, xf, yf, zf, d = _centres(p)
    ks = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
          if 1 <= kx * kx + ky * ky <= kmax * kmax]
    pick = rng.choice(len(ks), size=nmodes, replace=False)
    Ax = np.zeros((nz + 1, ny + 1, nx))      # at (x_i, y_{j-1/2}, z_{k-1/2})
    Ay = np.zeros((nz + 1, ny, nx + 1))      # at (x_{i-1/2}, y_j, z_{k-1/2})
    xe = np.concatenate([xf, [xf[-1] + d[0]]])
    ye = np.concatenate([yf, [yf[-1] + d[1]]])
    zs = np.concatenate([zf])                 # nz+1 wall-to-wall face heights
    for idx in pick:
        kx, ky = ks[idx]
        for comp in (0, 1):
            a = rng.normal()
            phi = rng.uniform(0.0, 2.0 * math.pi)
            m = int(rng.integers(1, 3))
            sz = np.sin(m * math.pi * zs)
            sz[0] = 0.0
            sz[-1] = 0.0
            if comp == 0:
                X, Y = np.meshgrid(xc, ye, indexing="xy")
                Ax += a * np.cos(2 * np.pi * (kx * X + ky * Y) + phi)[None] * sz[:, None, None]
            else:
                X, Y = np.meshgrid(xe, yc, indexing="xy")
                Ay += a * np.cos(2 * np.pi * (kx * X + ky * Y) + phi)[None] * sz[:, None, None]
    # B = curl A with A_z = 0: Bx = -dAy/dz, By = dAx/dz, Bz = dAy/dx - dAx/dy
    Bx = -(Ay[1:, :, :nx] - Ay[:-1, :, :nx]) / d[2]
    By = (Ax[1:, :ny, :] - Ax[:-1, :ny, :]) / d[2]
    Bz = (Ay[:, :, 1:] - Ay[:, :, :nx]) / d[0] - (Ax[:, 1:, :] - Ax[:, :ny, :]) / d[1]
    bx, by, bz = _cell_field(p, Bx, By, Bz)
    scale = math.sqrt(2.0 * P.mean() / (beta * np.mean(bx * bx + by * by + bz * bz)))
    return Bx * scale, By * scale, Bz * scale


# --------------------------------------------------------------------------
# Gas + radiation boxes
# --------------------------------------------------------------------------

def gasrad_params(nx, ny, nz, **kw):
    q = dict(eos=EOS_GASRAD, mu=0.6, rgas=R_CODE, arad=A_CODE)
    q.update(kw)
    return base_params(nx, ny, nz, **q)


def _tri(s):
    """Unit triangle wave with values uniformly distributed in [-1, 1]."""
    f = s - np.floor(s)
    return 4.0 * np.abs(f - 0.5) - 1.0


def gasrad_forward(p, rho, T):
    """Forward EOS values used only to set up inputs: e_int and P at (rho, T)
    for P = rho R T/mu + a T^4/3, e_int = R T/((gamma-1) mu) + a T^4/rho."""
    rmu = p["rgas"] / p["mu"]
    P = rho * rmu * T + p["arad"] * T ** 4 / 3.0
    e = rmu * T / (p["gamma"] - 1.0) + p["arad"] * T ** 4 / rho
    return P, e


def gasrad_box(n=256, seed=4, beta=1e6, cfl=0.4, steps=100):
    """Gas + radiation box on [0,1]^3, periodic: log10 rho = 2 tri(x + phi1),
    log10 T = 6.5 + 1.5 tri(y + phi2) (phases from seed), so rho and T are
    log-uniform over [1e-2, 1e2] and [1e5, 1e8] K; v = 0; uniform B_z with
    <2P>/B^2 = beta."""
    p = gasrad_params(n, n, n)
    xc, yc, zc, *_ = _centres(p)
    rng = np.random.default_rng(seed)
    ph1, ph2 = rng.uniform(0.0, 1.0, size=2)
    shp = (n, n, n)
    rho = np.broadcast_to((10.0 ** (2.0 * _tri(xc + ph1)))[None, None, :], shp).copy()
    T = np.broadcast_to((10.0 ** (6.5 + 1.5 * _tri(yc + ph2)))[None, :, None], shp).copy()
    P, e = gasrad_forward(p, rho, T)
    b0 = math.sqrt(2.0 * P.mean() / beta)
    Bx = np.zeros(shp)
    By = np.zeros(shp)
    Bz = np.full(shp, b0)
    zero = np.zeros(shp)
    U = _conserved(p, rho, zero, zero, zero, P, Bx, By, Bz, eint=e)
    return Workload("gasrad_box", p, U, Bx, By, Bz, T=T, cfl=cfl, steps=steps)


def eos_samples(n, seed=6, rho_range=(1e-2, 1e2), t_range=(1e5, 1e8)):
    """iid log-uniform (rho, T) samples."""
    rng = np.random.default_rng(seed)
    lr = rng.uniform(math.log10(rho_range[0]), math.log10(rho_range[1]), size=n)
    lt = rng.uniform(math.log10(t_range[0]), math.log10(t_range[1]), size=n)
    return 10.0 ** lr, 10.0 ** lt


def turbulence_box(n=384, seed=3, mach=3.0, beta=1.0, rho0=1e-2, T0=1e7, cfl=0.4, steps=100,
                   forcing=True):
    """Periodic gas+radiation MHD turbulence box on [0,1]^3: uniform rho0,
    T0 and B0 z_hat with 2 P0 / B0^2 = beta; a solenoidal velocity over the
    32 integer wavevectors with 1 <= |k| <= 2 (random amplitudes projected
    perpendicular to k, seed), scaled to rms Mach `mach`; a constant forcing
    acceleration with the same pattern and amplitude u_rms^2 / L, given as
    the 32 Fourier modes (k, a, phase), from which the library and the
    oracle each evaluate it.  The background is the uniform state (rho0,
    P0, gamma_e0, gamma_c0)."""
    p = gasrad_params(n, n, n)
    xc, yc, zc, *_ = _centres(p)
    rng = np.random.default_rng(seed)
    ks = [(a, b, c) for a in range(-2, 3) for b in range(-2, 3) for c in range(-2, 3)
          if 1 <= a * a + b * b + c * c <= 4]
    shp = (n, n, n)
    # v_c = sum_k a_c cos(2 pi k.x + phi) = Re sum_kz e^{2 pi i kz z} G_c,kz(y, x)
    # with G_c,kz = sum_{kx,ky} a_c e^{i phi} e^{2 pi i (kx x + ky y)}: one
    # real matrix product per component instead of a cosine per mode and cell
    G = np.zeros((3, 5, n, n), dtype=complex)
    ex = {m: np.exp(2j * np.pi * m * xc) for m in range(-2, 3)}
    ey = {m: np.exp(2j * np.pi * m * yc) for m in range(-2, 3)}
    modes = []
    for k in ks:
        kv = np.array(k, dtype=float)
        a = rng.normal(size=3)
        a = a - kv * (kv @ a) / (kv @ kv)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        modes.append([k[0], k[1], k[2], a[0], a[1], a[2], phi])
        plane = np.exp(1j * phi) * np.outer(ey[k[1]], ex[k[0]])
        for c in range(3):
            G[c, k[2] + 2] += a[c] * plane
    ez = np.stack([np.exp(2j * np.pi * m * zc) for m in range(-2, 3)], axis=1)  # [n, 5]
    lhs = np.concatenate([ez.real, -ez.imag], axis=1)                          # [n, 10]
    v = np.empty((3,) + shp)
    for c in range(3):
        rhs = np.concatenate([G[c].real.reshape(5, -1), G[c].imag.reshape(5, -1)], axis=0)
        v[c] = (lhs @ rhs).reshape(shp)
    rho = np.full(shp, rho0)
    T = np.full(shp, T0)
    P, e = gasrad_forward(p, rho, T)
    P0 = float(P.flat[0])
    # sound speed of the uniform state from the same thermodynamic identity
    rmu = p["rgas"] / p["mu"]
    cv = rmu / (p["gamma"] - 1.0) + 4.0 * p["arad"] * T0 ** 3 / rho0
    dpdT = rho0 * rmu + 4.0 * p["arad"] * T0 ** 3 / 3.0
    cs2 = rmu * T0 + T0 * dpdT * dpdT / (rho0 * rho0 * cv)
    urms = math.sqrt(float(np.mean(np.sum(v * v, axis=0))))
    v *= mach * math.sqrt(cs2) / urms
    # the forcing pattern is the raw velocity pattern, scaled to rms u_rms^2/L
    fscale = (mach * math.sqrt(cs2)) ** 2 / 1.0 / urms
    b0 = math.sqrt(2.0 * P0 / beta)
    Bx = np.zeros(shp)
    By = np.zeros(shp)
    Bz = np.full(shp, b0)
    U = _conserved(p, rho, v[0], v[1], v[2], P, Bx, By, Bz, eint=e)
    e0 = float(e.flat[0])
    ge0 = P0 / (rho0 * e0) + 1.0
    gc0 = rho0 * cs2 / P0
    bg_cc = np.array([[rho0] * n, [P0] * n, [ge0] * n, [gc0] * n])
    bg_fz = bg_cc.copy()
    fmodes = None
    if forcing:
        fmodes = np.array(modes, dtype=np.float64)
        fmodes[:, 3:6] *= fscale
    return Workload("turbulence_box", p, U, Bx, By, Bz, T=T, bg_cc=bg_cc, bg_fz=bg_fz,
                    fmodes=fmodes, cfl=cfl, steps=steps)


# --------------------------------------------------------------------------
# named benchmark configurations
# --------------------------------------------------------------------------

def config(idx: int, n: int | None = None):
    """The five workload configurations: 0 = 2D Orszag-Tang 64^2; 1 =
    stratified box 256^3; 2 = stratified box 512^3 with heating/cooling;
    3 = gas+radiation box 256^3; 4 = turbulence box 384^3.  n overrides the
    linear size (for scaled-down runs)."""
    if idx == 0:
        return orszag_tang(n or 64)
    if idx == 1:
        return stratified_box(n or 256, steps=100)
    if idx == 2:
        return stratified_box(n or 512, heating=True, steps=50)
    if idx == 3:
        return gasrad_box(n or 256)
    if idx == 4:
        return turbulence_box(n or 384)
    raise ValueError(idx)


def add_species(w, ns, seed=9, kmax=2, contrast=0.9):
    """The workload with ns passive species (Sect. 2.9): smooth positive mass
    fractions X_l = f_l / sum_m f_m, f_l = 1 + contrast x (a few random low
    Fourier modes, scaled into [-1, 1]), so they sum to one; U gains the rows
    rho X_l after its five fluid rows."""
    p = dict(w.params, nspecies=int(ns))
    xc, yc, zc, *_ = _centres(p)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    rng = np.random.default_rng(seed)
    f = np.empty((ns,) + X.shape)
    for l in range(ns):
        g = np.zeros_like(X)
        for _ in range(3):
            k = rng.integers(-kmax, kmax + 1, size=3)
            g += rng.normal() * np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z)
                                       + rng.uniform(0, 2 * np.pi))
        g /= max(np.abs(g).max(), 1e-300)
        f[l] = 1.0 + contrast * g
    Xl = f / f.sum(axis=0)
    U = np.ascontiguousarray(np.concatenate([w.U[:5], w.U[0][None] * Xl], axis=0))
    return Workload(w.name + f"+{ns}sp", p, U, w.Bx, w.By, w.Bz, T=w.T, bg_cc=w.bg_cc,
                    bg_fz=w.bg_fz, heat=w.heat, fmodes=w.fmodes, cfl=w.cfl, steps=w.steps)


def smooth_box(nx, ny, nz, seed=7, bcz=BC_PERIODIC, amp_v=0.3, amp_b=0.4, kmax=2, eos=EOS_IDEAL,
               blast=None):
    """Smooth random state on [0,1]^3 (parity tests on ragged grids): rho and
    P = 1 + 0.2 x (sum of a few low Fourier modes), v likewise with
    amplitude amp_v, face B from a random edge vector potential (amplitude
    amp_b) so that div B = 0 to round-off.  With a reflecting z the vector
    potential's x/y components vanish on the walls.  blast = (factor,
    radius): the thermal pressure is raised by that factor inside a sphere
    about the box centre (gas+radiation: T by factor^(1/4)), a pressure
    jump for the shock-flattening tests."""
    if eos == EOS_GASRAD:
        p = gasrad_params(nx, ny, nz, bcz=bcz)
    else:
        p = base_params(nx, ny, nz, bcz=bcz)
    rng = np.random.default_rng(seed)
    xc, yc, zc, xf, yf, zf, d = _centres(p)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")

    def field(scale):
        f = np.zeros_like(X)
        for _ in range(4):
            k = rng.integers(-kmax, kmax + 1, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            kz = k[2] if bcz == BC_PERIODIC else 0
            f += rng.normal() * np.cos(2 * np.pi * (k[0] * X + k[1] * Y + kz * Z) + ph)
        return scale * f / 4.0

    rho = 1.0 + np.abs(field(0.2)) + 0.05
    P = 1.0 + np.abs(field(0.2)) + 0.05
    v = [field(amp_v) for _ in range(3)]
    inside = None
    if blast is not None:
        inside = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2 < blast[1] ** 2
        P = np.where(inside, P * blast[0], P)
    if bcz == BC_REFLECT:
        v[2] *= np.sin(np.pi * Z)
    nzf = nz + 1 if bcz == BC_REFLECT else nz
    # edge vector potential on (x_i / x_{i-1/2}, y, z_{k-1/2}) positions
    def ax_at(Xe, Ye, Ze, wall):
        f = np.zeros_like(Xe)
        for _ in range(3):
            k = rng.integers(-kmax, kmax + 1, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            if bcz == BC_PERIODIC:
                f += rng.normal() * np.cos(2 * np.pi * (k[0] * Xe + k[1] * Ye + k[2] * Ze) + ph)
            else:
                f += rng.normal() * np.cos(2 * np.pi * (k[0] * Xe + k[1] * Ye) + ph) * \
                    np.sin(np.pi * max(1, abs(int(k[2]))) * Ze)
        if bcz == BC_REFLECT and wall:
            f[0] = 0.0
            f[-1] = 0.0
        return amp_b * f
    xe = np.concatenate([xf, [xf[-1] + d[0]]])
    ye = np.concatenate([yf, [yf[-1] + d[1]]])
    ze = np.concatenate([zf, [zf[-1] + d[2]]]) if bcz == BC_PERIODIC else zf
    # A_x at (x_i, y_{j-1/2}, z_{k-1/2}); A_y at (x_{i-1/2}, y_j, z_{k-1/2});
    # A_z at (x_{i-1/2}, y_{j-1/2}, z_k)
    Ze1, Ye1, Xe1 = np.meshgrid(ze, ye, xc, indexing="ij")
    Ax = ax_at(Xe1, Ye1, Ze1, True)
    Ze2, Ye2, Xe2 = np.meshgrid(ze, yc, xe, indexing="ij")
    Ay = ax_at(Xe2, Ye2, Ze2, True)
    Ze3, Ye3, Xe3 = np.meshgrid(zc, ye, xe, indexing="ij")
    Az = ax_at(Xe3, Ye3, Ze3, False)
    if bcz == BC_PERIODIC:
        # periodic images: last edge equals the first
        Ax[-1] = Ax[0]; Ax[:, -1] = Ax[:, 0]
        Ay[-1] = Ay[0]; Ay[:, :, -1] = Ay[:, :, 0]
        Az[:, -1] = Az[:, 0]; Az[:, :, -1] = Az[:, :, 0]
    Bx = (Az[:, 1:, :nx] - Az[:, :ny, :nx]) / d[1] - (Ay[1:nz + 1, :, :nx] - Ay[:nz, :, :nx]) / d[2]
    By = (Ax[1:nz + 1, :ny, :] - Ax[:nz, :ny, :]) / d[2] - (Az[:, :ny, 1:] - Az[:, :ny, :nx]) / d[0]
    Bz = (Ay[:nzf, :, 1:] - Ay[:nzf, :, :nx]) / d[0] - (Ax[:nzf, 1:, :] - Ax[:nzf, :ny, :]) / d[1]
    Bx, By, Bz = (np.ascontiguousarray(a) for a in (Bx, By, Bz))
    T = None
    eint = None
    if eos == EOS_GASRAD:
        T = 10.0 ** (6.0 + field(1.0))
        rho = 10.0 ** field(1.0)
        if inside is not None:
            T = np.where(inside, T * blast[0] ** 0.25, T)
        P, eint = gasrad_forward(p, rho, T)
        cs = np.sqrt(P.mean() / rho.mean())
        v = [vv * cs for vv in v]
        bx, by, bz = _cell_field(p, Bx, By, Bz)
        s = math.sqrt(2.0 * P.mean() / (10.0 * np.mean(bx * bx + by * by + bz * bz)))
        Bx, By, Bz = Bx * s, By * s, Bz * s
    U = _conserved(p, rho, v[0], v[1], v[2], P, Bx, By, Bz, eint=eint)
    return Workload("smooth_box", p, U, Bx, By, Bz, T=T)
