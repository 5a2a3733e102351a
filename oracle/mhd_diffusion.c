/*
 * mhd_diffusion.c -- plain FP64 CPU oracle of the thermal-diffusion
 * operator and its RKL2 super-time-stepping (arXiv 2604.12672, Sect. 2.10).
 *
 * TEST INFRASTRUCTURE ONLY (as mhd_oracle.c): loaded by the tests, never by
 * the product library, and sharing no source with the HIP path.
 *
 * The operator, in the paper's order:
 *   1. T per cell from (rho, e_int) with the EOS inversion (Sect. 2.2);
 *   2. chi = T^3 / (kappa rho) per cell with an opacity law
 *      kappa = kappa0 rho^alpha T^beta (READING: the paper takes tabulated
 *      or fitted opacities that are not available here; a power law stands
 *      in for them);
 *   3. face conductivity K = (4 a c / 3) * harmonic mean of chi (eq. after
 *      the thermal flux);
 *   4. face flux F = -K (T_R - T_L) / dx, zero through a reflecting wall;
 *   5. M[T] = (1/rho) * (F_lower - F_upper) / dx summed over the axes, the
 *      right-hand side of rho de/dt = div(K grad T) (eq. diffusion_eint).
 * RKL2 (Meyer, Balsara & Aslam) advances e_int over dt in s stages with the
 * published coefficients; the temperature form (paper: M -> M / c_v with
 * c_v frozen at the start) advances T instead and takes e_int from the
 * forward EOS at the end.  Only E changes: by rho (e_int_new - e_int_old).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mhd_oracle.h"

static size_t at(const orc_cfg *c, int i, int j, int k) {
  return ((size_t)k * c->ny + j) * c->nx + i;
}

static int wrapn(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

/* specific internal energy of cell q from U and the face field */
static double cell_eint(const orc_cfg *c, const double *U, const double *Bx,
                        const double *By, const double *Bz, int i, int j, int k) {
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  const size_t q = at(c, i, j, k);
  const double rho = U[q];
  const double vx = U[n + q] / rho, vy = U[2 * n + q] / rho, vz = U[3 * n + q] / rho;
  const double bx = 0.5 * (Bx[q] + Bx[at(c, wrapn(i + 1, c->nx), j, k)]);
  const double by = 0.5 * (By[q] + By[at(c, i, wrapn(j + 1, c->ny), k)]);
  const int kp = c->bcz == ORC_BC_REFLECT ? k + 1 : wrapn(k + 1, c->nz);
  const double bz = 0.5 * (Bz[q] + Bz[at(c, i, j, kp)]);
  return (U[4 * n + q] - 0.5 * rho * (vx * vx + vy * vy + vz * vz) -
          0.5 * (bx * bx + by * by + bz * bz)) / rho;
}

static double chi_of(const orc_opacity *op, double rho, double T) {
  const double kappa = op->kappa0 * pow(rho, op->alpha) * pow(T, op->beta);
  return T * T * T / (kappa * rho);
}

int orc_diffusion_rhs(const orc_cfg *c, const orc_opacity *op, const double *rho,
                      const double *T, double *M) {
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  const double pref = 4.0 * c->arad * op->clight / 3.0;
  const int nn[3] = {nx, ny, nz};
  const double dxs[3] = {c->dx, c->dy, c->dz};
#pragma omp parallel for collapse(3) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t q = at(c, i, j, k);
        const double chic = chi_of(op, rho[q], T[q]);
        double div = 0.0;
        for (int s = 0; s < 3; ++s) {
          if (nn[s] == 1) continue;
          const int ci[3] = {i, j, k};
          double flux[2];
          for (int side = 0; side < 2; ++side) { /* 0: lower face, 1: upper */
            int nb[3] = {ci[0], ci[1], ci[2]};
            nb[s] += side ? 1 : -1;
            if (s == 2 && c->bcz == ORC_BC_REFLECT && (nb[2] < 0 || nb[2] >= nz)) {
              flux[side] = 0.0; /* insulating wall */
              continue;
            }
            nb[s] = wrapn(nb[s], nn[s]);
            const size_t qn = at(c, nb[0], nb[1], nb[2]);
            const double chin = chi_of(op, rho[qn], T[qn]);
            const double K = pref * 2.0 * chic * chin / (chic + chin);
            /* flux through the face, positive along +s */
            flux[side] = side ? -K * (T[qn] - T[q]) / dxs[s] : -K * (T[q] - T[qn]) / dxs[s];
          }
          div += (flux[0] - flux[1]) / dxs[s];
        }
        M[q] = div / rho[q];
      }
  return ORC_OK;
}

int orc_parabolic_dt(const orc_cfg *c, const orc_opacity *op, const double *rho,
                     const double *T, double *dtp) {
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  const int nn[3] = {c->nx, c->ny, c->nz};
  const double dxs[3] = {c->dx, c->dy, c->dz};
  double smax = 0.0;
  for (size_t q = 0; q < n; ++q) {
    double P, e, cv, cs2;
    orc_eos_thermo(c, rho[q], T[q], &P, &e, &cv, &cs2);
    const double kappa = op->kappa0 * pow(rho[q], op->alpha) * pow(T[q], op->beta);
    const double D = 4.0 * c->arad * op->clight * T[q] * T[q] * T[q] /
                     (3.0 * kappa * rho[q] * rho[q] * cv);
    double sum = 0.0;
    for (int s = 0; s < 3; ++s)
      if (nn[s] > 1) sum += D / (dxs[s] * dxs[s]);
    if (sum > smax) smax = sum;
  }
  *dtp = 0.5 / smax;
  return ORC_OK;
}

int orc_rkl2_nsts(double dt_h, double dt_p) {
  const int s = 1 + (int)floor(0.5 * (sqrt(9.0 + 16.0 * dt_h / dt_p) - 1.0));
  return s > 3 ? s : 3;
}

/* RKL2 coefficients of stage j (1 <= j <= s):
   b_0 = b_1 = b_2 = 1/3, b_j = (j^2 + j - 2) / (2 j (j + 1)), a_j = 1 - b_j,
   w1 = 4 / (s^2 + s - 2); stage 1: mut = b_1 w1; stage j >= 2:
   mu = (2j - 1)/j b_j/b_{j-1}, nu = -(j - 1)/j b_j/b_{j-2}, mut = mu w1,
   gamt = -a_{j-1} mut. */
static double rkl2_b(int j) {
  if (j <= 2) return 1.0 / 3.0;
  return ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
}

void orc_rkl2_coeffs(int s, int j, double *mu, double *nu, double *mut, double *gamt) {
  const double w1 = 4.0 / ((double)s * s + s - 2.0);
  if (j == 1) {
    *mu = 0.0;
    *nu = 0.0;
    *mut = rkl2_b(1) * w1;
    *gamt = 0.0;
    return;
  }
  const double bj = rkl2_b(j), bj1 = rkl2_b(j - 1), bj2 = rkl2_b(j - 2);
  *mu = (2.0 * j - 1.0) / j * bj / bj1;
  *nu = -(j - 1.0) / j * bj / bj2;
  *mut = *mu * w1;
  *gamt = -(1.0 - bj1) * (*mut);
}

static int invert_all(const orc_cfg *c, const double *rho, const double *e, const double *tg,
                      double *T, size_t n) {
  int err = ORC_OK;
#pragma omp parallel for schedule(static) reduction(min : err)
  for (size_t q = 0; q < n; ++q) {
    int it, fb;
    const int rc = orc_eos_invert(c, rho[q], e[q], tg[q], &T[q], &it, &fb);
    if (rc < err) err = rc;
  }
  return err;
}

int orc_diffuse(const orc_cfg *c, const orc_opacity *op, double *U, const double *Bx,
                const double *By, const double *Bz, double *T, double dt, int nsts,
                int mode) {
  /* w1 = 4 / (s^2 + s - 2) needs s >= 2 */
  if (c->eos != ORC_EOS_GASRAD || !(dt > 0.0) || nsts < 2) return ORC_ERR_ARG;
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  double *rho = malloc(sizeof(double) * n), *e0 = malloc(sizeof(double) * n);
  double *y1 = malloc(sizeof(double) * n), *y2 = malloc(sizeof(double) * n);
  double *yn = malloc(sizeof(double) * n), *M0 = malloc(sizeof(double) * n);
  double *M = malloc(sizeof(double) * n), *Tw = malloc(sizeof(double) * n);
  double *cv0 = malloc(sizeof(double) * n);
  int err = ORC_OK;
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        const size_t q = at(c, i, j, k);
        rho[q] = U[q];
        e0[q] = cell_eint(c, U, Bx, By, Bz, i, j, k);
      }
  /* T^(0) from the EOS (guess: the caller's T) */
  err = invert_all(c, rho, e0, T, Tw, n);
  if (err) goto done;
  for (size_t q = 0; q < n; ++q) {
    double P, e, cv, cs2;
    orc_eos_thermo(c, rho[q], Tw[q], &P, &e, &cv, &cs2);
    cv0[q] = cv;
  }
  orc_diffusion_rhs(c, op, rho, Tw, M0);
  /* Y_0: e_int (mode 0) or T (mode 1); the stage operator is M, or M / c_v0 */
  const int tform = mode == 1;
  double *y0 = tform ? malloc(sizeof(double) * n) : e0;
  if (tform) {
    for (size_t q = 0; q < n; ++q) {
      y0[q] = Tw[q];
      M0[q] /= cv0[q];
    }
  }
  double mu, nu, mut, gamt;
  orc_rkl2_coeffs(nsts, 1, &mu, &nu, &mut, &gamt);
  for (size_t q = 0; q < n; ++q) {
    y2[q] = y0[q];
    y1[q] = y0[q] + mut * dt * M0[q];
  }
  for (int s = 2; s <= nsts; ++s) {
    /* temperature of Y_{s-1} */
    if (tform) {
      memcpy(Tw, y1, sizeof(double) * n);
    } else {
      err = invert_all(c, rho, y1, Tw, Tw, n);
      if (err) break;
    }
    orc_diffusion_rhs(c, op, rho, Tw, M);
    if (tform)
      for (size_t q = 0; q < n; ++q) M[q] /= cv0[q];
    orc_rkl2_coeffs(nsts, s, &mu, &nu, &mut, &gamt);
    for (size_t q = 0; q < n; ++q)
      yn[q] = mu * y1[q] + nu * y2[q] + (1.0 - mu - nu) * y0[q] + mut * dt * M[q] +
              gamt * dt * M0[q];
    double *t = y2;
    y2 = y1;
    y1 = yn;
    yn = t;
  }
  if (!err) {
    /* new e_int and T; E changes by rho (e_new - e_old) */
    for (size_t q = 0; q < n; ++q) {
      double enew, Tn;
      if (tform) {
        double P, cv, cs2;
        Tn = y1[q];
        orc_eos_thermo(c, rho[q], Tn, &P, &enew, &cv, &cs2);
      } else {
        int it, fb;
        enew = y1[q];
        const int rc = orc_eos_invert(c, rho[q], enew, Tw[q], &Tn, &it, &fb);
        if (rc < err) err = rc;
      }
      U[4 * n + q] += rho[q] * (enew - e0[q]);
      T[q] = Tn;
    }
  }
  if (tform) free(y0);
done:
  free(rho);
  free(e0);
  free(y1);
  free(y2);
  free(yn);
  free(M0);
  free(M);
  free(Tw);
  free(cv0);
  return err;
}
