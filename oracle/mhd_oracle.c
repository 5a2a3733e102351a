/*
 * mhd_oracle.c -- plain FP64 CPU oracle of one explicit finite-volume MHD
 * step of the PHLEGETHON scheme (arXiv 2604.12672, Sect. 2).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.  It is
 * written to be read against the paper, not to be fast: full-size scratch
 * arrays, explicit ghost cells, one loop per step of the algorithm.
 *
 * One evaluation of the spatial residual R(U) (eq. spatres) takes these
 * steps, in the paper's order:
 *   1. cons -> prim and the EOS inversion T(rho, e_int) per cell (Sect. 2.2),
 *      then the auxiliary indices gamma_e, gamma_c (Sect. 2.6);
 *   2. the deviation Delta W = W - W_hat from the background (Sect. 2.8);
 *   3. ghost cells: periodic copies, or mirror images at a reflecting wall
 *      (normal velocity and normal field odd, everything else even);
 *   4. per face: van Leer or PPH reconstruction of Delta W (Sect. 2.5), the
 *      background added back at the face, the HLLD/LHLLD flux (Sect. 2.6),
 *      and the equilibrium flux F_hat = F(W_hat_f, W_hat_f) subtracted
 *      (eq. wb1);
 *   5. Contact-CT edge EMFs (Sect. 2.4, Gardiner & Stone 2005);
 *   6. flux divergence minus (S - S_hat) (eqs. fv, wb2) and the face
 *      residual (1/A_f) sum_d l_d E_d (eq. induction).
 * The SSP-RK stages (Sect. 2.9) combine residuals; the CFL step follows
 * eq. cfl.  Readings of points the paper leaves open are marked READING.
 *
 * Compiled with -ffp-contract=off so every expression rounds as written.
 */
#include "mhd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 2 /* ghost layers: the 3-cell stencil (q = 1) needs two        */
#define NWF 10 /* rho, vx, vy, vz, P, bx, by, bz, gamma_e, gamma_c        */
enum { W_RHO, W_VX, W_VY, W_VZ, W_P, W_BX, W_BY, W_BZ, W_GE, W_GC };
enum { F_MASS, F_MN, F_MT1, F_MT2, F_EN, F_BT1, F_BT2, NFLUX };

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Equation of state (Sect. 2.2)                                        */
/* ------------------------------------------------------------------ */

/* Gas + radiation: P = rho R T / mu + a T^4 / 3,
   e_int = R T / ((gamma-1) mu) + a T^4 / rho  (eqs. prad, erad).
   c_s^2 = (dP/drho)_T + T (dP/dT)_rho^2 / (rho^2 c_v)  (READING: the paper
   does not print c_s for this EOS; this is the thermodynamic identity). */
int orc_eos_thermo(const orc_cfg *c, double rho, double T, double *P,
                   double *eint, double *cv, double *cs2) {
  if (c->eos == ORC_EOS_IDEAL) {
    /* ideal gas with e_int = c_v T and c_v = 1/(gamma-1) (T in units of
       P/rho); only used by tests */
    double cvv = 1.0 / (c->gamma - 1.0);
    *P = rho * T;
    *eint = cvv * T;
    *cv = cvv;
    *cs2 = c->gamma * T;
    return ORC_OK;
  }
  double rmu = c->rgas / c->mu;
  double T3 = T * T * T;
  double T4 = T3 * T;
  double p = rho * rmu * T + c->arad * T4 / 3.0;
  double e = rmu * T / (c->gamma - 1.0) + c->arad * T4 / rho;
  double cvv = rmu / (c->gamma - 1.0) + 4.0 * c->arad * T3 / rho;
  double dpdrho = rmu * T;
  double dpdT = rho * rmu + 4.0 * c->arad * T3 / 3.0;
  *P = p;
  *eint = e;
  *cv = cvv;
  *cs2 = dpdrho + T * dpdT * dpdT / (rho * rho * cvv);
  return ORC_OK;
}

/* Newton-Raphson T <- T + delta_e / c_v from the guess, stopping when
   |delta_e| / e_int < eps is met before an update is applied (Sect. 2.2).
   e_int(T) = C_g T + (a/rho) T^4 is increasing and convex, so Newton from any
   positive guess converges; the bracketed solve below is reached only for a
   non-finite or non-positive guess or when the iteration cap is hit.
   READING: bracket T_lo = min(e/(2 C_g), (rho e/(2a))^(1/4)),
   T_hi = min(e/C_g, (rho e/a)^(1/4)): at the root one of the two positive
   terms is at least e/2 and neither exceeds e. */
int orc_eos_invert(const orc_cfg *c, double rho, double eint, double Tguess,
                   double *T, int *iters, int *fallback) {
  double cg = c->rgas / ((c->gamma - 1.0) * c->mu);
  double ar = c->arad / rho;
  double tol = c->newton_tol;
  *iters = 0;
  *fallback = 0;
  if (!(rho > 0.0) || !(eint > 0.0) || !isfinite(rho) || !isfinite(eint))
    return ORC_ERR_UNPHYSICAL;
  double t = Tguess;
  if (isfinite(t) && t > 0.0) {
    for (int n = 0; n < c->newton_maxit; ++n) {
      double t3 = t * t * t;
      double de = eint - (cg * t + ar * t3 * t);
      if (fabs(de) < tol * eint) {
        *T = t;
        *iters = n;
        return ORC_OK;
      }
      double cv = cg + 4.0 * ar * t3;
      t = t + de / cv;
      *iters = n + 1;
      if (!(isfinite(t) && t > 0.0)) break;
    }
  }
  /* bracketed Newton-bisection */
  *fallback = 1;
  double lo = fmin(eint / (2.0 * cg), pow(eint / (2.0 * ar), 0.25));
  double hi = fmin(eint / cg, pow(eint / ar, 0.25));
  t = 0.5 * (lo + hi);
  for (int n = 0; n < 400; ++n) {
    double t3 = t * t * t;
    double de = eint - (cg * t + ar * t3 * t);
    if (fabs(de) < tol * eint) {
      *T = t;
      return ORC_OK;
    }
    if (de > 0.0)
      lo = t;
    else
      hi = t;
    double tn = t + de / (cg + 4.0 * ar * t3);
    if (tn > lo && tn < hi)
      t = tn;
    else
      t = 0.5 * (lo + hi);
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * hi) {
      *T = t;
      return ORC_OK;
    }
  }
  return ORC_ERR_EOS;
}

/* Primitive state of one cell from its conserved variables, with the cell
   field B_cc = mean of the two faces per axis (READING). */
static int cons2prim(const orc_cfg *c, const double u[5], const double bcc[3],
                     double tguess, double *tout, double *w) {
  double rho = u[0];
  if (!(rho > 0.0) || !isfinite(rho)) return ORC_ERR_UNPHYSICAL;
  double vx = u[1] / rho, vy = u[2] / rho, vz = u[3] / rho;
  double b2 = bcc[0] * bcc[0] + bcc[1] * bcc[1] + bcc[2] * bcc[2];
  double eint = (u[4] - 0.5 * rho * (vx * vx + vy * vy + vz * vz) - 0.5 * b2) /
                rho;
  if (!(eint > 0.0) || !isfinite(eint)) return ORC_ERR_UNPHYSICAL;
  double P, cs2;
  if (c->eos == ORC_EOS_IDEAL) {
    P = (c->gamma - 1.0) * rho * eint;
    cs2 = c->gamma * P / rho;
  } else {
    double T, e2, cv;
    int it, fb;
    int rc = orc_eos_invert(c, rho, eint, tguess, &T, &it, &fb);
    if (rc) return rc;
    orc_eos_thermo(c, rho, T, &P, &e2, &cv, &cs2);
    if (tout) *tout = T;
  }
  if (!(P > 0.0)) return ORC_ERR_UNPHYSICAL;
  w[W_RHO] = rho;
  w[W_VX] = vx;
  w[W_VY] = vy;
  w[W_VZ] = vz;
  w[W_P] = P;
  w[W_BX] = bcc[0];
  w[W_BY] = bcc[1];
  w[W_BZ] = bcc[2];
  /* auxiliary indices (Sect. 2.6): gamma_e = P/(rho e_int) + 1,
     gamma_c = rho c_s^2 / P */
  w[W_GE] = P / (rho * eint) + 1.0;
  w[W_GC] = rho * cs2 / P;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Reconstruction (Sect. 2.5)                                           */
/* ------------------------------------------------------------------ */

/* READING: the van Leer (1974) limiter in its harmonic form,
   slope = 2ab/(a+b) when a and b have the same sign, else 0. */
double orc_vanleer(double a, double b) {
  double ab = a * b;
  if (ab > 0.0) return 2.0 * ab / (a + b);
  return 0.0;
}

/* READING: the paper's PPH reconstructs every primitive except the mass
   fractions with an unlimited parabola on the three-cell stencil (q = 1);
   without species that is the parabola whose averages over the cells
   i-1, i, i+1 are the cell values, evaluated at the two faces of cell i:
   w(i+1/2) = (-w_{i-1} + 5 w_i + 2 w_{i+1}) / 6,
   w(i-1/2) = (2 w_{i-1} + 5 w_i - w_{i+1}) / 6. */
void orc_pph(double wm, double wc, double wp, double *lo, double *hi) {
  *hi = (-wm + 5.0 * wc + 2.0 * wp) / 6.0;
  *lo = (2.0 * wm + 5.0 * wc - wp) / 6.0;
}

/* READING: the paper reconstructs mass fractions with a limited parabola in
   PPH mode and cites the limiter; here each face value of the three-cell
   parabola is first bounded by the two averages beside that face, then the
   parabola is made monotone inside the cell with the constraints of
   Colella & Woodward (1984): a cell holding a local extremum is flat, and a
   face value that would make the parabola overshoot inside the cell is
   moved so the parabola's extremum sits at the opposite face. */
static double clamp2(double v, double a, double b) {
  const double lo = a < b ? a : b, hi = a < b ? b : a;
  return v < lo ? lo : (v > hi ? hi : v);
}

void orc_pph_limited(double wm, double wc, double wp, double *lo, double *hi) {
  double l, h;
  orc_pph(wm, wc, wp, &l, &h);
  l = clamp2(l, wm, wc);
  h = clamp2(h, wc, wp);
  if ((h - wc) * (wc - l) <= 0.0) {
    l = wc;
    h = wc;
  } else {
    const double d = h - l;
    const double m6 = 6.0 * (wc - 0.5 * (l + h));
    if (d * m6 > d * d)
      l = 3.0 * wc - 2.0 * h;
    else if (-d * d > d * m6)
      h = 3.0 * wc - 2.0 * l;
  }
  *lo = l;
  *hi = h;
}

/* ------------------------------------------------------------------ */
/* HLLD / LHLLD Riemann solver (Sect. 2.6; Miyoshi & Kusano 2005)       */
/* ------------------------------------------------------------------ */

typedef struct {
  double rho, vn, vt1, vt2, P, bt1, bt2;
  double ptot, E, cf, cs;
  double U[NFLUX], F[NFLUX];
} side_t;

static void side_setup(const double *W, double bn, side_t *s) {
  s->rho = W[0];
  s->vn = W[1];
  s->vt1 = W[2];
  s->vt2 = W[3];
  s->P = W[4];
  s->bt1 = W[5];
  s->bt2 = W[6];
  double ge = W[7], gc = W[8];
  /* e_int and c_s from the reconstructed indices (Sect. 2.6) */
  double eint = s->P / (s->rho * (ge - 1.0));
  double cs2 = gc * s->P / s->rho;
  double b2 = bn * bn + s->bt1 * s->bt1 + s->bt2 * s->bt2;
  double v2 = s->vn * s->vn + s->vt1 * s->vt1 + s->vt2 * s->vt2;
  s->ptot = s->P + 0.5 * b2;
  s->E = s->rho * eint + 0.5 * s->rho * v2 + 0.5 * b2;
  s->cs = sqrt(cs2);
  /* fast magnetosonic speed along the normal; READING: the discriminant is
     clipped at zero against rounding */
  double a2b2 = cs2 + b2 / s->rho;
  double disc = a2b2 * a2b2 - 4.0 * cs2 * bn * bn / s->rho;
  if (disc < 0.0) disc = 0.0;
  s->cf = sqrt(0.5 * (a2b2 + sqrt(disc)));
  double vb = s->vn * bn + s->vt1 * s->bt1 + s->vt2 * s->bt2;
  s->U[F_MASS] = s->rho;
  s->U[F_MN] = s->rho * s->vn;
  s->U[F_MT1] = s->rho * s->vt1;
  s->U[F_MT2] = s->rho * s->vt2;
  s->U[F_EN] = s->E;
  s->U[F_BT1] = s->bt1;
  s->U[F_BT2] = s->bt2;
  /* ideal-MHD flux along the normal (Sect. 2.1) */
  s->F[F_MASS] = s->rho * s->vn;
  s->F[F_MN] = s->rho * s->vn * s->vn + s->ptot - bn * bn;
  s->F[F_MT1] = s->rho * s->vn * s->vt1 - bn * s->bt1;
  s->F[F_MT2] = s->rho * s->vn * s->vt2 - bn * s->bt2;
  s->F[F_EN] = (s->E + s->ptot) * s->vn - bn * vb;
  s->F[F_BT1] = s->vn * s->bt1 - bn * s->vt1;
  s->F[F_BT2] = s->vn * s->bt2 - bn * s->vt2;
}

/* Single-star state of one side: U*_a from S_a, S_M, p_T* (MK05 sect. 4). */
static void star_state(const side_t *s, double S, double SM, double pst,
                       double bn, double *Us, double *vst1, double *vst2,
                       double *bst1, double *bst2) {
  double rst = s->rho * (S - s->vn) / (S - SM);
  double den = s->rho * (S - s->vn) * (S - SM) - bn * bn;
  double v1, v2, b1, b2;
  /* READING: degenerate when |den| <= 1e-8 rho (S - v_n)^2; then the
     transverse velocity and field pass through unchanged */
  if (fabs(den) <= 1e-8 * s->rho * (S - s->vn) * (S - s->vn)) {
    v1 = s->vt1;
    v2 = s->vt2;
    b1 = s->bt1;
    b2 = s->bt2;
  } else {
    double fv = bn * (SM - s->vn) / den;
    double fb = (s->rho * (S - s->vn) * (S - s->vn) - bn * bn) / den;
    v1 = s->vt1 - s->bt1 * fv;
    v2 = s->vt2 - s->bt2 * fv;
    b1 = s->bt1 * fb;
    b2 = s->bt2 * fb;
  }
  double vb = s->vn * bn + s->vt1 * s->bt1 + s->vt2 * s->bt2;
  double vbs = SM * bn + v1 * b1 + v2 * b2;
  double Est = ((S - s->vn) * s->E - s->ptot * s->vn + pst * SM +
                bn * (vb - vbs)) /
               (S - SM);
  Us[F_MASS] = rst;
  Us[F_MN] = rst * SM;
  Us[F_MT1] = rst * v1;
  Us[F_MT2] = rst * v2;
  Us[F_EN] = Est;
  Us[F_BT1] = b1;
  Us[F_BT2] = b2;
  *vst1 = v1;
  *vst2 = v2;
  *bst1 = b1;
  *bst2 = b2;
}

/* Low-dissipation factor xi on the upwind part of p_T* (Sect. 2.6, eq.
   pstar).  READING: the paper states only xi ~ max(M_L, M_R) applied below
   M = 0.6; the default is the continuous xi = min(1, max(M_L,M_R)/0.6),
   with the sonic Mach number M = |v| / c_s. */
static double xi_factor(const orc_cfg *c, const side_t *L, const side_t *R) {
  if (c->xi_mode == ORC_XI_OFF) return 1.0;
  double vL = sqrt(L->vn * L->vn + L->vt1 * L->vt1 + L->vt2 * L->vt2);
  double vR = sqrt(R->vn * R->vn + R->vt1 * R->vt1 + R->vt2 * R->vt2);
  double M = fmax(vL / L->cs, vR / R->cs);
  if (c->xi_mode == ORC_XI_STEP) return M < c->mach_cut ? M : 1.0;
  return fmin(1.0, M / c->mach_cut);
}

int orc_riemann(const orc_cfg *c, const double *WL, const double *WR,
                double bn, double *flux) {
  side_t L, R;
  side_setup(WL, bn, &L);
  side_setup(WR, bn, &R);
  /* fastest-wave estimates (MK05 eq. 67) */
  double cmax = fmax(L.cf, R.cf);
  double SL = fmin(L.vn, R.vn) - cmax;
  double SR = fmax(L.vn, R.vn) + cmax;
  /* region selection, eq. flux-hlld, with its tie-breaks as printed */
  if (0.0 <= SL) {
    memcpy(flux, L.F, sizeof(L.F));
    return ORC_OK;
  }
  if (SR < 0.0) {
    memcpy(flux, R.F, sizeof(R.F));
    return ORC_OK;
  }
  double aL = (SL - L.vn) * L.rho, aR = (SR - R.vn) * R.rho;
  double den = aR - aL;
  /* contact speed and star total pressure; xi scales the dissipative term */
  double SM = (aR * R.vn - aL * L.vn - R.ptot + L.ptot) / den;
  double xi = xi_factor(c, &L, &R);
  double pst = (aR * L.ptot - aL * R.ptot +
                xi * L.rho * R.rho * (SR - R.vn) * (SL - L.vn) * (R.vn - L.vn)) /
               den;
  double UsL[NFLUX], UsR[NFLUX];
  double vL1, vL2, bL1, bL2, vR1, vR2, bR1, bR2;
  star_state(&L, SL, SM, pst, bn, UsL, &vL1, &vL2, &bL1, &bL2);
  star_state(&R, SR, SM, pst, bn, UsR, &vR1, &vR2, &bR1, &bR2);
  double sqL = sqrt(UsL[F_MASS]), sqR = sqrt(UsR[F_MASS]);
  double SsL = SM - fabs(bn) / sqL;
  double SsR = SM + fabs(bn) / sqR;
  double FsL[NFLUX], FsR[NFLUX];
  for (int q = 0; q < NFLUX; ++q) {
    FsL[q] = L.F[q] + SL * (UsL[q] - L.U[q]);
    FsR[q] = R.F[q] + SR * (UsR[q] - R.U[q]);
  }
  /* READING: the interface pressure p_T* carries the low-dissipation factor
     into the normal-momentum flux, rho* S_M^2 + p_T* - B_n^2 (identical to
     F + S (U* - U) when xi = 1).  The energy flux needs no change: E* above
     already contains p_T*, and the double-star states share rho* S_M. */
  FsL[F_MN] = UsL[F_MASS] * SM * SM + pst - bn * bn;
  FsR[F_MN] = UsR[F_MASS] * SM * SM + pst - bn * bn;
  if (SL < 0.0 && 0.0 <= SsL) {
    memcpy(flux, FsL, sizeof(FsL));
    return ORC_OK;
  }
  if (SsR < 0.0 && 0.0 <= SR) {
    memcpy(flux, FsR, sizeof(FsR));
    return ORC_OK;
  }
  /* double-star states (MK05 sect. 4.3) */
  double sg = bn >= 0.0 ? 1.0 : -1.0;
  double isum = 1.0 / (sqL + sqR);
  double v1 = (sqL * vL1 + sqR * vR1 + (bR1 - bL1) * sg) * isum;
  double v2 = (sqL * vL2 + sqR * vR2 + (bR2 - bL2) * sg) * isum;
  double b1 = (sqL * bR1 + sqR * bL1 + sqL * sqR * (vR1 - vL1) * sg) * isum;
  double b2 = (sqL * bR2 + sqR * bL2 + sqL * sqR * (vR2 - vL2) * sg) * isum;
  double vbss = SM * bn + v1 * b1 + v2 * b2;
  double vbsL = SM * bn + vL1 * bL1 + vL2 * bL2;
  double vbsR = SM * bn + vR1 * bR1 + vR2 * bR2;
  double UssL[NFLUX], UssR[NFLUX];
  UssL[F_MASS] = UsL[F_MASS];
  UssL[F_MN] = UsL[F_MN];
  UssL[F_MT1] = UsL[F_MASS] * v1;
  UssL[F_MT2] = UsL[F_MASS] * v2;
  UssL[F_EN] = UsL[F_EN] - sqL * (vbsL - vbss) * sg;
  UssL[F_BT1] = b1;
  UssL[F_BT2] = b2;
  UssR[F_MASS] = UsR[F_MASS];
  UssR[F_MN] = UsR[F_MN];
  UssR[F_MT1] = UsR[F_MASS] * v1;
  UssR[F_MT2] = UsR[F_MASS] * v2;
  UssR[F_EN] = UsR[F_EN] + sqR * (vbsR - vbss) * sg;
  UssR[F_BT1] = b1;
  UssR[F_BT2] = b2;
  if (SsL < 0.0 && 0.0 <= SM) {
    for (int q = 0; q < NFLUX; ++q) flux[q] = FsL[q] + SsL * (UssL[q] - UsL[q]);
    return ORC_OK;
  }
  for (int q = 0; q < NFLUX; ++q) flux[q] = FsR[q] + SsR * (UssR[q] - UsR[q]);
  return ORC_OK;
}

/* HLL (Harten, Lax & van Leer 1983), the two-wave solver of flattened
   cells (Sect. 2.7): one intermediate state between the fastest waves,
   F = (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L), upwind
   outside the fan; the wave speeds are those of orc_riemann. */
int orc_hll(const orc_cfg *c, const double *WL, const double *WR, double bn,
            double *flux) {
  (void)c;
  side_t L, R;
  side_setup(WL, bn, &L);
  side_setup(WR, bn, &R);
  double cmax = fmax(L.cf, R.cf);
  double SL = fmin(L.vn, R.vn) - cmax;
  double SR = fmax(L.vn, R.vn) + cmax;
  if (0.0 <= SL) {
    memcpy(flux, L.F, sizeof(L.F));
    return ORC_OK;
  }
  if (SR < 0.0) {
    memcpy(flux, R.F, sizeof(R.F));
    return ORC_OK;
  }
  for (int q = 0; q < NFLUX; ++q)
    flux[q] = (SR * L.F[q] - SL * R.F[q] + SL * SR * (R.U[q] - L.U[q])) / (SR - SL);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                         */
/* ------------------------------------------------------------------ */

typedef struct {
  int nx, ny, nz, nzf;
  int gx, gy, gz; /* padded extents (NG ghosts each side)            */
  size_t gcells;
} grid_t;

static void grid_init(const orc_cfg *c, grid_t *g) {
  g->nx = c->nx;
  g->ny = c->ny;
  g->nz = c->nz;
  g->nzf = c->bcz == ORC_BC_REFLECT ? c->nz + 1 : c->nz;
  g->gx = c->nx + 2 * NG;
  g->gy = c->ny + 2 * NG;
  g->gz = c->nz + 2 * NG;
  g->gcells = (size_t)g->gx * g->gy * g->gz;
}

/* padded index of (i,j,k), each in [-NG, n+NG) */
static inline size_t gidx(const grid_t *g, int i, int j, int k) {
  return ((size_t)(k + NG) * g->gy + (j + NG)) * g->gx + (i + NG);
}
static inline size_t cidx(const grid_t *g, int i, int j, int k) {
  return ((size_t)k * g->ny + j) * g->nx + i;
}
static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

/* z index of the interior cell that supplies ghost plane k, and whether the
   image is mirrored (reflecting wall) */
static inline int zsrc(const orc_cfg *c, int k, int *mirror) {
  int nz = c->nz;
  *mirror = 0;
  if (k >= 0 && k < nz) return k;
  if (c->bcz == ORC_BC_PERIODIC) return wrap(k, nz);
  *mirror = 1;
  return k < 0 ? -1 - k : 2 * nz - 1 - k;
}

static double bg_cell(const orc_cfg *c, int f, int k) {
  if (!c->bg_cc) return 0.0;
  return c->bg_cc[(size_t)f * c->nz + k];
}
static double bg_face(const orc_cfg *c, int f, int k) {
  if (!c->bg_fz) return 0.0;
  int nzf = c->bcz == ORC_BC_REFLECT ? c->nz + 1 : c->nz;
  return c->bg_fz[(size_t)f * nzf + k];
}

/* cell-centred field: mean of the two faces on each axis */
static void cell_field(const orc_cfg *c, const grid_t *g, const double *Bx,
                       const double *By, const double *Bz, int i, int j, int k,
                       double b[3]) {
  int ip = wrap(i + 1, g->nx), jp = wrap(j + 1, g->ny);
  int kp = c->bcz == ORC_BC_REFLECT ? k + 1 : wrap(k + 1, g->nz);
  b[0] = 0.5 * (Bx[cidx(g, i, j, k)] + Bx[cidx(g, ip, j, k)]);
  b[1] = 0.5 * (By[cidx(g, i, j, k)] + By[cidx(g, i, jp, k)]);
  b[2] = 0.5 * (Bz[cidx(g, i, j, k)] + Bz[cidx(g, i, j, kp)]);
}

/* ------------------------------------------------------------------ */
/* Shock flattening (Sect. 2.7)                                         */
/* ------------------------------------------------------------------ */

/* Flags from the thermal pressure P [nz][ny][nx] of every cell.
   Detector: (|P_{i+1} - P_{i-1}| + |P_{j+1} - P_{j-1}| + |P_{k+1} - P_{k-1}|)
   / (eps_SF P) > 1, the neighbours taken periodically in x and y and in a
   periodic z, and as mirror images at a reflecting wall (P is even, so the
   image of cell 0 below the wall is cell 0 itself).  Every cell within the
   5x5x5 cube (two cells per axis) of a detected cell is flagged; across a
   wall the cube is cut off (a mirror image only repeats cells inside it). */
static void shock_flags_from_p(const orc_cfg *c, const grid_t *g, const double *P,
                               unsigned char *flags) {
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const size_t n = (size_t)nx * ny * nz;
  unsigned char *det = (unsigned char *)malloc(n);
#pragma omp parallel for collapse(3) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int mir;
        const int km = zsrc(c, k - 1, &mir), kp = zsrc(c, k + 1, &mir);
        const double sum =
            fabs(P[cidx(g, wrap(i + 1, nx), j, k)] - P[cidx(g, wrap(i - 1, nx), j, k)]) +
            fabs(P[cidx(g, i, wrap(j + 1, ny), k)] - P[cidx(g, i, wrap(j - 1, ny), k)]) +
            fabs(P[cidx(g, i, j, kp)] - P[cidx(g, i, j, km)]);
        det[cidx(g, i, j, k)] = sum / (c->eps_sf * P[cidx(g, i, j, k)]) > 1.0;
      }
#pragma omp parallel for collapse(3) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        unsigned char f = 0;
        for (int dk = -2; dk <= 2; ++dk) {
          int kk = k + dk;
          if (c->bcz == ORC_BC_REFLECT) {
            if (kk < 0 || kk >= nz) continue;
          } else {
            kk = wrap(kk, nz);
          }
          for (int dj = -2; dj <= 2; ++dj)
            for (int di = -2; di <= 2; ++di)
              f |= det[cidx(g, wrap(i + di, nx), wrap(j + dj, ny), kk)];
        }
        flags[cidx(g, i, j, k)] = f;
      }
  free(det);
}

int orc_shock_flags(const orc_cfg *c, const double *U, const double *Bx,
                    const double *By, const double *Bz, const double *Tguess,
                    unsigned char *flags) {
  grid_t g;
  grid_init(c, &g);
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  double *P = (double *)malloc(sizeof(double) * n);
  int err = ORC_OK;
#pragma omp parallel for collapse(3) schedule(static) reduction(min : err)
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        const size_t q = cidx(&g, i, j, k);
        double u[5], b[3], w[NWF], t = 0.0;
        for (int f = 0; f < 5; ++f) u[f] = U[f * n + q];
        cell_field(c, &g, Bx, By, Bz, i, j, k, b);
        const int rc = cons2prim(c, u, b, Tguess ? Tguess[q] : 0.0, &t, w);
        if (rc < err) err = rc;
        P[q] = w[W_P];
      }
  if (!err) shock_flags_from_p(c, &g, P, flags);
  free(P);
  return err;
}

int orc_primitives(const orc_cfg *c, const double *U, const double *Bx,
                   const double *By, const double *Bz, const double *Tguess,
                   double *Tout, double *out) {
  grid_t g;
  grid_init(c, &g);
  size_t n = (size_t)g.nx * g.ny * g.nz;
  int err = ORC_OK;
#pragma omp parallel for collapse(3) schedule(static) reduction(min : err)
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        size_t q = cidx(&g, i, j, k);
        double u[5], b[3], w[NWF], t = 0.0;
        for (int f = 0; f < 5; ++f) u[f] = U[f * n + q];
        cell_field(c, &g, Bx, By, Bz, i, j, k, b);
        int rc = cons2prim(c, u, b, Tguess ? Tguess[q] : 0.0, &t, w);
        if (rc < err) err = rc;
        for (int f = 0; f < NWF; ++f) out[f * n + q] = rc ? NAN : w[f];
        if (Tout) Tout[q] = t;
      }
  return err;
}

/* ------------------------------------------------------------------ */
/* Spatial residual                                                     */
/* ------------------------------------------------------------------ */

/* face-frame component order: axis d has normal d, t1 = d+1, t2 = d+2 */
static const int vel_of[3][3] = {
    {W_VX, W_VY, W_VZ}, {W_VY, W_VZ, W_VX}, {W_VZ, W_VX, W_VY}};
static const int fld_of[3][3] = {
    {W_BX, W_BY, W_BZ}, {W_BY, W_BZ, W_BX}, {W_BZ, W_BX, W_BY}};
/* conserved momentum slot (1..3) of v_n, v_t1, v_t2 */
static const int mom_of[3][3] = {{1, 2, 3}, {2, 3, 1}, {3, 1, 2}};

typedef struct {
  /* flux minus equilibrium flux, 7 components, on the padded grid */
  double *F[NFLUX];
  double *mass; /* mass flux before the subtraction (contact direction) */
} faceflux_t;

static void wb_flux(const orc_cfg *c, double rho, double P, double ge,
                    double gc, double *Fh) {
  /* equilibrium flux F_hat = F(W_hat_f, W_hat_f) from the same solver
     (eq. wb1 and the consistency argument after it) */
  double W[9] = {rho, 0.0, 0.0, 0.0, P, 0.0, 0.0, ge, gc};
  if (rho > 0.0 && P > 0.0)
    orc_riemann(c, W, W, 0.0, Fh);
  else
    for (int q = 0; q < NFLUX; ++q) Fh[q] = 0.0;
}

int orc_residual(const orc_cfg *c, const double *U, const double *Bx,
                 const double *By, const double *Bz, const double *Tguess,
                 double *Tout, double *RU, double *RBx, double *RBy,
                 double *RBz) {
  grid_t g;
  grid_init(c, &g);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const size_t n = (size_t)nx * ny * nz;
  const size_t G = g.gcells;
  const double dxs[3] = {c->dx, c->dy, c->dz};
  int err = ORC_OK;

  /* steps 1-2: primitives and their deviation from the background; the
     mass fractions X_l = (rho X_l) / rho of the passive species */
  const int nsp = c->nspecies;
  if (nsp < 0 || nsp > 64) return ORC_ERR_ARG;
  double *dW = (double *)malloc(sizeof(double) * NWF * G);
  double *Xs = nsp ? (double *)malloc(sizeof(double) * nsp * G) : NULL;
  double *Tnew = (double *)malloc(sizeof(double) * n);
  double *Pc = (double *)malloc(sizeof(double) * n); /* thermal P per cell */
#pragma omp parallel for collapse(3) schedule(static) reduction(min : err)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t q = cidx(&g, i, j, k);
        double u[5], b[3], w[NWF], t = 0.0;
        for (int f = 0; f < 5; ++f) u[f] = U[f * n + q];
        cell_field(c, &g, Bx, By, Bz, i, j, k, b);
        int rc = cons2prim(c, u, b, Tguess ? Tguess[q] : 0.0, &t, w);
        if (rc < err) err = rc;
        Tnew[q] = t;
        Pc[q] = w[W_P];
        for (int l = 0; l < nsp; ++l)
          Xs[(size_t)l * G + gidx(&g, i, j, k)] = U[(5 + l) * n + q] / u[0];
        /* Delta W = W - W_hat (Sect. 2.8); the background has zero velocity
           and field, so only rho, P, gamma_e, gamma_c change */
        w[W_RHO] -= bg_cell(c, 0, k);
        w[W_P] -= bg_cell(c, 1, k);
        w[W_GE] -= bg_cell(c, 2, k);
        w[W_GC] -= bg_cell(c, 3, k);
        size_t p = gidx(&g, i, j, k);
        for (int f = 0; f < NWF; ++f) dW[f * G + p] = w[f];
      }
  if (err) {
    free(dW);
    free(Xs);
    free(Tnew);
    free(Pc);
    return err;
  }
  if (Tout) memcpy(Tout, Tnew, sizeof(double) * n);
  free(Tnew);

  /* shock flattening (Sect. 2.7): flags of the stage's input state on the
     padded grid, ghosts filled like the primitives below (a mirror image
     carries the flag of its source cell) */
  unsigned char *flg = NULL;
  if (c->flatten) {
    unsigned char *fi = (unsigned char *)malloc(n);
    shock_flags_from_p(c, &g, Pc, fi);
    flg = (unsigned char *)calloc(G, 1);
    for (int k = -NG; k < nz + NG; ++k) {
      int mir;
      const int ks = zsrc(c, k, &mir);
      for (int j = -NG; j < ny + NG; ++j)
        for (int i = -NG; i < nx + NG; ++i)
          flg[gidx(&g, i, j, k)] = fi[cidx(&g, wrap(i, nx), wrap(j, ny), ks)];
    }
    free(fi);
  }
  free(Pc);

  /* step 3: ghost cells -- x and y periodic; z periodic or mirrored */
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = -NG; i < nx + NG; ++i) {
        if (i >= 0 && i < nx) continue;
        size_t d = gidx(&g, i, j, k), s = gidx(&g, wrap(i, nx), j, k);
        for (int f = 0; f < NWF; ++f) dW[f * G + d] = dW[f * G + s];
        for (int l = 0; l < nsp; ++l) Xs[(size_t)l * G + d] = Xs[(size_t)l * G + s];
      }
  for (int k = 0; k < nz; ++k)
    for (int j = -NG; j < ny + NG; ++j) {
      if (j >= 0 && j < ny) continue;
      for (int i = -NG; i < nx + NG; ++i) {
        size_t d = gidx(&g, i, j, k), s = gidx(&g, i, wrap(j, ny), k);
        for (int f = 0; f < NWF; ++f) dW[f * G + d] = dW[f * G + s];
        for (int l = 0; l < nsp; ++l) Xs[(size_t)l * G + d] = Xs[(size_t)l * G + s];
      }
    }
  for (int k = -NG; k < nz + NG; ++k) {
    if (k >= 0 && k < nz) continue;
    int mir;
    int ks = zsrc(c, k, &mir);
    for (int j = -NG; j < ny + NG; ++j)
      for (int i = -NG; i < nx + NG; ++i) {
        size_t d = gidx(&g, i, j, k), s = gidx(&g, i, j, ks);
        for (int f = 0; f < NWF; ++f) {
          double v = dW[f * G + s];
          /* mirror image at a wall: v_z and B_z flip sign (Table bcs,
             reflecting: zero normal velocity and normal field) */
          if (mir && (f == W_VZ || f == W_BZ)) v = -v;
          dW[f * G + d] = v;
        }
        /* mass fractions are even across a wall */
        for (int l = 0; l < nsp; ++l) Xs[(size_t)l * G + d] = Xs[(size_t)l * G + s];
      }
  }

  /* equilibrium fluxes: x/y faces sit at cell-centre heights, z faces at
     face heights */
  double *Fh_c = (double *)malloc(sizeof(double) * NFLUX * nz);
  double *Fh_f = (double *)malloc(sizeof(double) * NFLUX * g.nzf);
  for (int k = 0; k < nz; ++k)
    wb_flux(c, bg_cell(c, 0, k), bg_cell(c, 1, k), bg_cell(c, 2, k),
            bg_cell(c, 3, k), Fh_c + NFLUX * k);
  for (int k = 0; k < g.nzf; ++k)
    wb_flux(c, bg_face(c, 0, k), bg_face(c, 1, k), bg_face(c, 2, k),
            bg_face(c, 3, k), Fh_f + NFLUX * k);

  /* step 4: fluxes on every face the update and the edge EMFs need.
     Face (i,j,k) of axis d is the lower face of cell (i,j,k) along d. */
  faceflux_t FF[3];
  double *FX[3] = {NULL, NULL, NULL}; /* species fluxes [ns][G] per axis */
  for (int d = 0; d < 3; ++d) {
    for (int q = 0; q < NFLUX; ++q) {
      FF[d].F[q] = (double *)malloc(sizeof(double) * G);
    }
    FF[d].mass = (double *)malloc(sizeof(double) * G);
    if (nsp) FX[d] = (double *)malloc(sizeof(double) * nsp * G);
  }
  for (int d = 0; d < 3; ++d) {
    int lo[3] = {-1, -1, -1}, hi[3] = {nx, ny, nz};
    lo[d] = 0; /* faces 0..n along the normal, cells -1..n across */
    const int ds[3] = {d == 0, d == 1, d == 2};
    const size_t st = (size_t)ds[0] + (size_t)ds[1] * g.gx +
                      (size_t)ds[2] * g.gx * g.gy;
    int ferr = ORC_OK;
#pragma omp parallel for collapse(3) schedule(static) reduction(min : ferr)
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          size_t pR = gidx(&g, i, j, k); /* cell on the upper side */
          size_t pL = pR - st;           /* cell on the lower side */
          /* reconstructed quantities: rho, v_n, v_t1, v_t2, P, B_t1, B_t2,
             gamma_e, gamma_c (Sect. 2.5, 2.6; the normal field is the face
             value and is not reconstructed) */
          const int fl[9] = {W_RHO,        vel_of[d][0], vel_of[d][1],
                             vel_of[d][2], W_P,          fld_of[d][1],
                             fld_of[d][2], W_GE,         W_GC};
          /* flattened cells: van Leer reconstruction, and the HLL solver
             on every face that touches one (Sect. 2.7) */
          const int fL = flg ? flg[pL] : 0, fR = flg ? flg[pR] : 0;
          const int pphL = c->recon == ORC_RECON_PPH && !fL;
          const int pphR = c->recon == ORC_RECON_PPH && !fR;
          double WL[9], WR[9];
          for (int m = 0; m < 9; ++m) {
            const double *a = dW + (size_t)fl[m] * G;
            double unused;
            if (pphL) {
              orc_pph(a[pL - st], a[pL], a[pR], &unused, &WL[m]);
            } else {
              double sL = orc_vanleer(a[pL] - a[pL - st], a[pR] - a[pL]);
              WL[m] = a[pL] + 0.5 * sL; /* Delta W_{i-1/2, L} */
            }
            if (pphR) {
              orc_pph(a[pL], a[pR], a[pR + st], &WR[m], &unused);
            } else {
              double sR = orc_vanleer(a[pR] - a[pL], a[pR + st] - a[pR]);
              WR[m] = a[pR] - 0.5 * sR; /* Delta W_{i-1/2, R} */
            }
          }
          /* background at the face added back (Sect. 2.8) */
          double bh[4];
          const double *Fh;
          if (d == 2) {
            int kf = c->bcz == ORC_BC_REFLECT ? k : wrap(k, nz);
            for (int f = 0; f < 4; ++f) bh[f] = bg_face(c, f, kf);
            Fh = Fh_f + NFLUX * kf;
          } else {
            int mir;
            int kc = zsrc(c, k, &mir);
            for (int f = 0; f < 4; ++f) bh[f] = bg_cell(c, f, kc);
            Fh = Fh_c + NFLUX * kc;
          }
          WL[0] += bh[0];
          WR[0] += bh[0];
          WL[4] += bh[1];
          WR[4] += bh[1];
          WL[7] += bh[2];
          WR[7] += bh[2];
          WL[8] += bh[3];
          WR[8] += bh[3];
          /* normal field at the face */
          double bn;
          if (d == 0) {
            int mir;
            int kc = zsrc(c, k, &mir);
            bn = Bx[cidx(&g, wrap(i, nx), wrap(j, ny), kc)];
          } else if (d == 1) {
            int mir;
            int kc = zsrc(c, k, &mir);
            bn = By[cidx(&g, wrap(i, nx), wrap(j, ny), kc)];
          } else {
            int kf = c->bcz == ORC_BC_REFLECT ? k : wrap(k, nz);
            bn = Bz[cidx(&g, wrap(i, nx), wrap(j, ny), kf)];
          }
          double fx[NFLUX];
          if (!(WL[0] > 0.0 && WR[0] > 0.0 && WL[4] > 0.0 && WR[4] > 0.0)) {
            ferr = ORC_ERR_UNPHYSICAL;
            for (int q = 0; q < NFLUX; ++q) fx[q] = 0.0;
          } else if (fL || fR) {
            orc_hll(c, WL, WR, bn, fx);
          } else {
            orc_riemann(c, WL, WR, bn, fx);
          }
          FF[d].mass[pR] = fx[F_MASS];
          /* eq. wb1: F <- F - F_hat */
          for (int q = 0; q < NFLUX; ++q) FF[d].F[q][pR] = fx[q] - Fh[q];
          /* passive species (Sect. 2.9): face mass fractions reconstructed
             like the primitives (van Leer, or the limited parabola in PPH
             mode; van Leer in flattened cells), rescaled on each side so
             they sum to one, and carried by the mass flux from the upwind
             side (READING: the side of the contact that holds the face in
             HLLC / HLLD, i.e. the sign of the mass flux; the same rule on
             HLL faces), so the species fluxes add up to the mass flux */
          if (nsp) {
            double XL[64], XR[64], sL = 0.0, sR = 0.0;
            for (int l = 0; l < nsp; ++l) {
              const double *a = Xs + (size_t)l * G;
              double unused;
              if (pphL) {
                orc_pph_limited(a[pL - st], a[pL], a[pR], &unused, &XL[l]);
              } else {
                double sl = orc_vanleer(a[pL] - a[pL - st], a[pR] - a[pL]);
                XL[l] = a[pL] + 0.5 * sl;
              }
              if (pphR) {
                orc_pph_limited(a[pL], a[pR], a[pR + st], &XR[l], &unused);
              } else {
                double sr = orc_vanleer(a[pR] - a[pL], a[pR + st] - a[pR]);
                XR[l] = a[pR] - 0.5 * sr;
              }
              sL += XL[l];
              sR += XR[l];
            }
            const double m = fx[F_MASS];
            for (int l = 0; l < nsp; ++l)
              FX[d][(size_t)l * G + pR] = m >= 0.0 ? m * (XL[l] / sL) : m * (XR[l] / sR);
          }
        }
    if (ferr < err) err = ferr;
  }
  free(Fh_c);
  free(Fh_f);
  free(flg);
  if (err) goto done;

  {
    /* step 5: Contact-CT edge EMFs (Sect. 2.4; Gardiner & Stone 2005).
       Cell reference EMF E_ref = -(v x B_cc).  For E_c with a = c+1,
       b = c+2 (cyclic): faces of axis a carry E_c = -F_a[B_t1] and faces of
       axis b carry E_c = +F_b[B_t2] (t1, t2 of the face frame). */
    double *Eref[3], *Ed[3];
    for (int cc = 0; cc < 3; ++cc) {
      Eref[cc] = (double *)malloc(sizeof(double) * G);
      Ed[cc] = (double *)malloc(sizeof(double) * G);
    }
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = -NG; k < nz + NG; ++k)
      for (int j = -NG; j < ny + NG; ++j)
        for (int i = -NG; i < nx + NG; ++i) {
          size_t p = gidx(&g, i, j, k);
          double vx = dW[W_VX * G + p], vy = dW[W_VY * G + p],
                 vz = dW[W_VZ * G + p];
          double bx = dW[W_BX * G + p], by = dW[W_BY * G + p],
                 bz = dW[W_BZ * G + p];
          Eref[0][p] = -(vy * bz - vz * by);
          Eref[1][p] = -(vz * bx - vx * bz);
          Eref[2][p] = -(vx * by - vy * bx);
        }
    for (int cc = 0; cc < 3; ++cc) {
      const int a = (cc + 1) % 3, b = (cc + 2) % 3;
      /* offsets of one cell along a and along b */
      const size_t off[3] = {1, (size_t)g.gx, (size_t)g.gx * g.gy};
      const size_t sa = off[a], sb = off[b];
      /* edge E_c(i,j,k) sits at the lower a- and lower b- side of cell
         (i,j,k); its index runs 0..n along a and b, 0..n-1 along c */
      int hi[3] = {nx, ny, nz};
      hi[cc] -= 1;
#pragma omp parallel for collapse(3) schedule(static)
      for (int k = 0; k <= hi[2]; ++k)
        for (int j = 0; j <= hi[1]; ++j)
          for (int i = 0; i <= hi[0]; ++i) {
            size_t p = gidx(&g, i, j, k);
            /* a-faces at (a-1/2, b) and (a-1/2, b-1): E_c = -F_a[B_t1] */
            double Ea_b = -FF[a].F[F_BT1][p];
            double Ea_bm = -FF[a].F[F_BT1][p - sb];
            /* b-faces at (a, b-1/2) and (a-1, b-1/2): E_c = +F_b[B_t2] */
            double Eb_a = FF[b].F[F_BT2][p];
            double Eb_am = FF[b].F[F_BT2][p - sa];
            const double *Er = Eref[cc];
            double r_ab = Er[p], r_amb = Er[p - sa], r_abm = Er[p - sb],
                   r_ambm = Er[p - sa - sb];
            /* mass fluxes through the four faces set the upwind side */
            double m_ab = FF[a].mass[p], m_abm = FF[a].mass[p - sb];
            double m_ba = FF[b].mass[p], m_bam = FF[b].mass[p - sa];
            double d1, d2, d3, d4;
            /* (1) along b from the a-face at b: upwind in a */
            if (m_ab > 0.0)
              d1 = Eb_am - r_amb;
            else if (m_ab < 0.0)
              d1 = Eb_a - r_ab;
            else
              d1 = 0.5 * ((Eb_am - r_amb) + (Eb_a - r_ab));
            /* (2) along b from the a-face at b-1 */
            if (m_abm > 0.0)
              d2 = Eb_am - r_ambm;
            else if (m_abm < 0.0)
              d2 = Eb_a - r_abm;
            else
              d2 = 0.5 * ((Eb_am - r_ambm) + (Eb_a - r_abm));
            /* (3) along a from the b-face at a: upwind in b */
            if (m_ba > 0.0)
              d3 = Ea_bm - r_abm;
            else if (m_ba < 0.0)
              d3 = Ea_b - r_ab;
            else
              d3 = 0.5 * ((Ea_bm - r_abm) + (Ea_b - r_ab));
            /* (4) along a from the b-face at a-1 */
            if (m_bam > 0.0)
              d4 = Ea_bm - r_ambm;
            else if (m_bam < 0.0)
              d4 = Ea_b - r_amb;
            else
              d4 = 0.5 * ((Ea_bm - r_ambm) + (Ea_b - r_amb));
            /* READING: the corner value is the mean of the four face values
               each carried to the edge with the upwind cell-side gradient,
               E = 1/4 (sum of face EMFs) + 1/4 (d1 + d2 + d3 + d4), which
               reduces to the face EMF of a plane-parallel problem */
            double E = 0.25 * (Ea_b + Ea_bm + Eb_a + Eb_am) +
                       0.25 * (d1 + d2 + d3 + d4);
            /* a reflecting wall has no tangential EMF: the edges on it
               carry zero (v_z = 0 and B_z = 0 there) */
            if (c->bcz == ORC_BC_REFLECT && cc != 2 && (k == 0 || k == nz))
              E = 0.0;
            Ed[cc][p] = E;
          }
    }

    /* step 6: residuals.  Cells: flux divergence minus (S - S_hat). */
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          size_t p = gidx(&g, i, j, k), q = cidx(&g, i, j, k);
          const size_t off[3] = {1, (size_t)g.gx, (size_t)g.gx * g.gy};
          double r[5] = {0, 0, 0, 0, 0};
          for (int d = 0; d < 3; ++d) {
            const double *const *F = (const double *const *)FF[d].F;
            size_t pu = p + off[d];
            r[0] += (F[F_MASS][pu] - F[F_MASS][p]) / dxs[d];
            r[mom_of[d][0]] += (F[F_MN][pu] - F[F_MN][p]) / dxs[d];
            r[mom_of[d][1]] += (F[F_MT1][pu] - F[F_MT1][p]) / dxs[d];
            r[mom_of[d][2]] += (F[F_MT2][pu] - F[F_MT2][p]) / dxs[d];
            r[4] += (F[F_EN][pu] - F[F_EN][p]) / dxs[d];
          }
          /* sources (Sect. 2.1): S = (0, rho g, rho g.u + heating); the
             equilibrium source S_hat = (0, rho_hat g, 0) is subtracted
             (eq. wb2).  READING: heating and forcing are not part of S_hat,
             otherwise the deviation form would cancel them. */
          double rho = U[q], mx = U[n + q], my = U[2 * n + q],
                 mz = U[3 * n + q];
          double s[5] = {0, 0, 0, 0, 0};
          s[3] = (rho - bg_cell(c, 0, k)) * c->gz;
          s[4] = mz * c->gz;
          if (c->heat) s[4] += c->heat[k];
          if (c->force) {
            double fx = c->force[q], fy = c->force[n + q],
                   fz = c->force[2 * n + q];
            s[1] += rho * fx;
            s[2] += rho * fy;
            s[3] += rho * fz;
            s[4] += mx * fx + my * fy + mz * fz;
          }
          for (int f = 0; f < 5; ++f) RU[f * n + q] = r[f] - s[f];
          /* species: divergence of their fluxes (no sources) */
          for (int l = 0; l < nsp; ++l) {
            double rx = 0.0;
            for (int d = 0; d < 3; ++d) {
              const double *Fl = FX[d] + (size_t)l * G;
              rx += (Fl[p + off[d]] - Fl[p]) / dxs[d];
            }
            RU[(5 + l) * n + q] = rx;
          }
        }
    /* faces: R_f = (1/A_f) sum_d l_d E_d = (curl E)_n (eq. induction) */
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          size_t p = gidx(&g, i, j, k), q = cidx(&g, i, j, k);
          size_t sx = 1, sy = (size_t)g.gx, sz = (size_t)g.gx * g.gy;
          RBx[q] = (Ed[2][p + sy] - Ed[2][p]) / c->dy -
                   (Ed[1][p + sz] - Ed[1][p]) / c->dz;
          RBy[q] = (Ed[0][p + sz] - Ed[0][p]) / c->dz -
                   (Ed[2][p + sx] - Ed[2][p]) / c->dx;
        }
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = 0; k < g.nzf; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          size_t p = gidx(&g, i, j, k), q = cidx(&g, i, j, k);
          size_t sx = 1, sy = (size_t)g.gx;
          double r = (Ed[1][p + sx] - Ed[1][p]) / c->dx -
                     (Ed[0][p + sy] - Ed[0][p]) / c->dy;
          /* wall faces keep B_z = 0 */
          if (c->bcz == ORC_BC_REFLECT && (k == 0 || k == nz)) r = 0.0;
          RBz[q] = r;
        }
    for (int cc = 0; cc < 3; ++cc) {
      free(Eref[cc]);
      free(Ed[cc]);
    }
  }
done:
  for (int d = 0; d < 3; ++d) {
    for (int q = 0; q < NFLUX; ++q) free(FF[d].F[q]);
    free(FF[d].mass);
    free(FX[d]);
  }
  free(dW);
  free(Xs);
  return err;
}

/* ------------------------------------------------------------------ */
/* SSP-RK step (Sect. 2.9)                                              */
/* ------------------------------------------------------------------ */

/* U_out = a U0 + b Us - cdt R, element-wise */
static void combine(size_t n, double a, const double *U0, double b,
                    const double *Us, double cdt, const double *R,
                    double *out) {
#pragma omp parallel for schedule(static)
  for (long long q = 0; q < (long long)n; ++q)
    out[q] = a * U0[q] + b * Us[q] - cdt * R[q];
}

int orc_step(const orc_cfg *c, double *U, double *Bx, double *By, double *Bz,
             double *T, double dt) {
  grid_t g;
  grid_init(c, &g);
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const size_t nf = (size_t)g.nx * g.ny * g.nzf;
  /* one buffer holding U (with the species), Bx, By, Bz back to back */
  const size_t nu = (size_t)(5 + c->nspecies) * n;
  const size_t tot = nu + 2 * n + nf;
  double *S0 = (double *)malloc(sizeof(double) * tot);
  double *S1 = (double *)malloc(sizeof(double) * tot);
  double *R = (double *)malloc(sizeof(double) * tot);
  memcpy(S0, U, sizeof(double) * nu);
  memcpy(S0 + nu, Bx, sizeof(double) * n);
  memcpy(S0 + nu + n, By, sizeof(double) * n);
  memcpy(S0 + nu + 2 * n, Bz, sizeof(double) * nf);
  /* stage coefficients (a, b, c): U_new = a U^n + b U^(s) - c dt R(U^(s)) */
  static const double rk2[2][3] = {{0.0, 1.0, 1.0}, {0.5, 0.5, 0.5}};
  static const double rk3[3][3] = {
      {0.0, 1.0, 1.0}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};
  int ns = c->rk_order == 3 ? 3 : 2;
  const double(*co)[3] = c->rk_order == 3 ? rk3 : rk2;
  double *Tw = NULL;
  if (c->eos == ORC_EOS_GASRAD) Tw = T;
  int err = ORC_OK;
  const double *Us = S0;
  for (int s = 0; s < ns; ++s) {
    err = orc_residual(c, Us, Us + nu, Us + nu + n, Us + nu + 2 * n, Tw, Tw, R, R + nu,
                       R + nu + n, R + nu + 2 * n);
    if (err) break;
    combine(tot, co[s][0], S0, co[s][1], Us, co[s][2] * dt, R, S1);
    Us = S1;
  }
  if (!err) {
    memcpy(U, S1, sizeof(double) * nu);
    memcpy(Bx, S1 + nu, sizeof(double) * n);
    memcpy(By, S1 + nu + n, sizeof(double) * n);
    memcpy(Bz, S1 + nu + 2 * n, sizeof(double) * nf);
  }
  free(S0);
  free(S1);
  free(R);
  return err;
}

/* ------------------------------------------------------------------ */
/* CFL time step, eq. cfl                                               */
/* ------------------------------------------------------------------ */

int orc_compute_dt(const orc_cfg *c, const double *U, const double *Bx,
                   const double *By, const double *Bz, const double *T,
                   double cfl, double *dt) {
  grid_t g;
  grid_init(c, &g);
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const int nn[3] = {g.nx, g.ny, g.nz};
  const double dxs[3] = {c->dx, c->dy, c->dz};
  double smax = 0.0;
  int err = ORC_OK;
#pragma omp parallel for collapse(3) schedule(static) reduction(max : smax) \
    reduction(min : err)
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        size_t q = cidx(&g, i, j, k);
        double u[5], b[3], w[NWF], t;
        for (int f = 0; f < 5; ++f) u[f] = U[f * n + q];
        cell_field(c, &g, Bx, By, Bz, i, j, k, b);
        int rc = cons2prim(c, u, b, T ? T[q] : 0.0, &t, w);
        if (rc) {
          if (rc < err) err = rc;
          continue;
        }
        double rho = w[W_RHO];
        double a2 = w[W_GC] * w[W_P] / rho;
        double b2 = (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) / rho;
        double sum = 0.0;
        for (int s = 0; s < 3; ++s) {
          /* READING: an axis with a single cell carries no dynamics and
             is left out of the sum */
          if (nn[s] == 1) continue;
          double bs2 = b[s] * b[s] / rho;
          double disc = (a2 + b2) * (a2 + b2) - 4.0 * a2 * bs2;
          if (disc < 0.0) disc = 0.0;
          double cf = sqrt(0.5 * ((a2 + b2) + sqrt(disc)));
          sum += (fabs(w[W_VX + s]) + cf) / dxs[s];
        }
        if (sum > smax) smax = sum;
      }
  if (err) return err;
  *dt = cfl / smax;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Diagnostics                                                          */
/* ------------------------------------------------------------------ */

void orc_forcing(const orc_cfg *c, const double *modes, int nmodes, const double origin[3],
                 const double period[3], double *out) {
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  const double pi2 = 6.283185307179586476925286766559;
#pragma omp parallel for collapse(3) schedule(static)
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        const double X = (origin[0] + (i + 0.5) * c->dx) / period[0];
        const double Y = (origin[1] + (j + 0.5) * c->dy) / period[1];
        const double Z = (origin[2] + (k + 0.5) * c->dz) / period[2];
        double f[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < nmodes; ++m) {
          const double *md = modes + 7 * m;
          const double ph = pi2 * (md[0] * X + md[1] * Y + md[2] * Z) + md[6];
          const double cs = cos(ph);
          f[0] += md[3] * cs;
          f[1] += md[4] * cs;
          f[2] += md[5] * cs;
        }
        const size_t q = ((size_t)k * c->ny + j) * c->nx + i;
        out[q] = f[0];
        out[n + q] = f[1];
        out[2 * n + q] = f[2];
      }
}

void orc_divb(const orc_cfg *c, const double *Bx, const double *By,
              const double *Bz, double *out) {
  grid_t g;
  grid_init(c, &g);
#pragma omp parallel for collapse(3) schedule(static)
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        int ip = wrap(i + 1, g.nx), jp = wrap(j + 1, g.ny);
        int kp = c->bcz == ORC_BC_REFLECT ? k + 1 : wrap(k + 1, g.nz);
        out[cidx(&g, i, j, k)] =
            (Bx[cidx(&g, ip, j, k)] - Bx[cidx(&g, i, j, k)]) / c->dx +
            (By[cidx(&g, i, jp, k)] - By[cidx(&g, i, j, k)]) / c->dy +
            (Bz[cidx(&g, i, j, kp)] - Bz[cidx(&g, i, j, k)]) / c->dz;
      }
}
