/*
 * mhd_oracle.h -- plain FP64 CPU oracle for one explicit finite-volume MHD
 * step of the PHLEGETHON scheme (arXiv 2604.12672, Sect. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes this
 * header or links this code; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no source with the
 * HIP path.
 *
 * Grid and storage (all arrays FP64, x fastest, interior cells only):
 *   U   [5+ns][nz][ny][nx] rho, m_x, m_y, m_z, E (E includes |B_cc|^2/2),
 *                         then rho X_l of the ns passive species (Sect. 2.9)
 *   Bx  [nz][ny][nx]      face i holds B_x at x_{i-1/2}      (x periodic)
 *   By  [nz][ny][nx]      face j holds B_y at y_{j-1/2}      (y periodic)
 *   Bz  [nzf][ny][nx]     face k holds B_z at z_{k-1/2}; nzf = nz when z is
 *                         periodic, nz+1 when z is reflecting (walls at k=0,nz)
 *   T   [nz][ny][nx]      temperature (gas+radiation EOS only)
 * x and y are always periodic; z is periodic or reflecting.
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_UNPHYSICAL (-4)
#define ORC_ERR_EOS (-5)

#define ORC_BC_PERIODIC 0
#define ORC_BC_REFLECT 1

#define ORC_EOS_IDEAL 0
#define ORC_EOS_GASRAD 1

/* low-dissipation factor of the star-region pressure (Sect. 2.6, eq. pstar) */
#define ORC_XI_LINEAR 0  /* xi = min(1, max(M_L,M_R)/M_cut)                 */
#define ORC_XI_STEP 1    /* xi = max(M_L,M_R) if that is < M_cut, else 1    */
#define ORC_XI_OFF 2     /* xi = 1: plain HLLD                              */

/* reconstruction of the face states (Sect. 2.5) */
#define ORC_RECON_VANLEER 0 /* linear, van Leer limited slope                  */
#define ORC_RECON_PPH 1     /* piecewise parabolic (PPH without species): the
                               unlimited third-order parabola of the three-cell
                               stencil                                        */

typedef struct {
  int nx, ny, nz;
  double dx, dy, dz;
  int bcz;               /* ORC_BC_PERIODIC or ORC_BC_REFLECT              */
  int eos;               /* ORC_EOS_IDEAL or ORC_EOS_GASRAD                */
  double gamma;          /* adiabatic index of the gas                     */
  double mu, rgas, arad; /* gas+radiation EOS constants (code units)       */
  double gz;             /* constant gravitational acceleration along z    */
  int rk_order;          /* 2 or 3 (SSP-RK, Sect. 2.9)                     */
  double newton_tol;     /* relative residual bound of the T inversion     */
  int newton_maxit;      /* Newton iterations before the bracketed solve   */
  double mach_cut;       /* Mach threshold of the low-dissipation factor   */
  int xi_mode;           /* ORC_XI_*                                        */
  int recon;             /* ORC_RECON_*                                     */
  int flatten;           /* 1: shock flattening (Sect. 2.7), 0: off         */
  double eps_sf;         /* threshold epsilon_SF of the shock detector      */
  int nspecies;          /* passive species ns carried as rho X_l in U      */
  const double *bg_cc;   /* [4][nz]  background rho, P, gamma_e, gamma_c at
                            cell centres, or NULL for a zero background     */
  const double *bg_fz;   /* [4][nzf] the same at z faces (NULL with bg_cc)  */
  const double *heat;    /* [nz] energy source per volume, or NULL          */
  const double *force;   /* [3][nz][ny][nx] acceleration field, or NULL     */
} orc_cfg;

/* Forcing acceleration from Fourier modes (the driven-turbulence setup;
   not a step of the paper's scheme): at every cell centre x,
     f(x) = sum_m a_m cos(2 pi (k_m,x X + k_m,y Y + k_m,z Z) + phi_m),
   X = (origin[0] + (i + 1/2) dx) / period[0], likewise Y, Z, evaluated term
   by term.  modes [nmodes][7] = (k_x, k_y, k_z, a_x, a_y, a_z, phi) with
   integer wavenumbers; origin = position of the grid's first cell corner
   relative to the forcing's reference corner; period = the forcing's box
   lengths.  out [3][nz][ny][nx]. */
void orc_forcing(const orc_cfg *c, const double *modes, int nmodes, const double origin[3],
                 const double period[3], double *out);

/* Forward EOS at (rho, T): pressure, specific internal energy, c_v and the
   adiabatic sound speed squared (Sect. 2.2, eqs. prad/erad). */
int orc_eos_thermo(const orc_cfg *c, double rho, double T, double *P,
                   double *eint, double *cv, double *cs2);

/* Newton-Raphson inversion T(rho, e_int) from a guess (Sect. 2.2), with the
   bracketed Newton-bisection fallback.  iters = Newton steps taken,
   fallback = 1 when the bracketed solve produced the result. */
int orc_eos_invert(const orc_cfg *c, double rho, double eint, double Tguess,
                   double *T, int *iters, int *fallback);

/* Van Leer limited slope from the two one-sided differences (Sect. 2.5). */
double orc_vanleer(double a, double b);

/* PPH face values of a cell from its own and its neighbours' averages
   (Sect. 2.5): lo = value at the lower face, hi = at the upper face. */
void orc_pph(double wm, double wc, double wp, double *lo, double *hi);

/* Limited parabola of the mass fractions in PPH mode (Sect. 2.5): the
   face values of the three-cell parabola of orc_pph bounded by the averages
   beside each face, then made monotone inside the cell with the constraints
   of Colella & Woodward (1984). */
void orc_pph_limited(double wm, double wc, double wp, double *lo, double *hi);

/* HLLD / LHLLD interface flux (Sect. 2.6, eq. flux-hlld) in the face frame.
   W = {rho, v_n, v_t1, v_t2, P, B_t1, B_t2, gamma_e, gamma_c};
   flux = {mass, mom_n, mom_t1, mom_t2, energy, B_t1, B_t2}. */
int orc_riemann(const orc_cfg *c, const double *WL, const double *WR,
                double bn, double *flux);

/* HLL two-wave flux (Harten, Lax & van Leer 1983; the solver of flattened
   cells, Sect. 2.7) with the same wave-speed estimates as orc_riemann;
   same arguments and layout. */
int orc_hll(const orc_cfg *c, const double *WL, const double *WR, double bn,
            double *flux);

/* Shock-flattening flags of every cell (Sect. 2.7): the detector on the
   thermal pressure of the state, dilated over the 5x5x5 neighbourhood.
   flags [nz][ny][nx] = 1 (flattened) or 0.  Tguess as for orc_residual. */
int orc_shock_flags(const orc_cfg *c, const double *U, const double *Bx,
                    const double *By, const double *Bz, const double *Tguess,
                    unsigned char *flags);

/* Spatial residual R(U) of eq. spatres for cells and faces; dU/dt = -RU,
   dB/dt = -RB.  Tguess/Tout: EOS guess and result (gas+radiation only;
   Tout may alias Tguess). */
int orc_residual(const orc_cfg *c, const double *U, const double *Bx,
                 const double *By, const double *Bz, const double *Tguess,
                 double *Tout, double *RU, double *RBx, double *RBy,
                 double *RBz);

/* One SSP-RK step of size dt in place (Sect. 2.9).  T is the previous-step
   temperature guess on input and the last stage's solution on output. */
int orc_step(const orc_cfg *c, double *U, double *Bx, double *By, double *Bz,
             double *T, double dt);

/* Hyperbolic CFL time step, eq. cfl.  T is only read (as the EOS guess). */
int orc_compute_dt(const orc_cfg *c, const double *U, const double *Bx,
                   const double *By, const double *Bz, const double *T,
                   double cfl, double *dt);

/* Cell divergence of the face field, eq. divb. out [nz][ny][nx]. */
void orc_divb(const orc_cfg *c, const double *Bx, const double *By,
              const double *Bz, double *out);

/* Primitive state per cell: out [10][nz][ny][nx] = rho, v(3), P, B_cc(3),
   gamma_e, gamma_c; Tout may be NULL. */
int orc_primitives(const orc_cfg *c, const double *U, const double *Bx,
                   const double *By, const double *Bz, const double *Tguess,
                   double *Tout, double *out);

/* Number of OpenMP threads the oracle runs with (1 without OpenMP), and a
   setter for the following calls (n > 0). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* ------------------------------------------------------------------ */
/* Thermal diffusion and RKL2 super-time-stepping (Sect. 2.10),        */
/* mhd_diffusion.c                                                     */
/* ------------------------------------------------------------------ */

/* opacity law kappa = kappa0 rho^alpha T^beta; clight = speed of light in
   code units (the conductivity is K = (4 a c / 3) chi, chi = T^3/(kappa rho)) */
typedef struct {
  double kappa0, alpha, beta, clight;
} orc_opacity;

#define ORC_DIFF_EINT 0 /* evolve e_int, EOS inversion every stage          */
#define ORC_DIFF_TEMP 1 /* evolve T with c_v frozen at the start            */

/* M[T] = (1/rho) div(K grad T) per cell (rho, T, M: [nz][ny][nx]) */
int orc_diffusion_rhs(const orc_cfg *c, const orc_opacity *op, const double *rho,
                      const double *T, double *M);
/* parabolic limit dt_p = 1 / (2 max sum_s D / dx_s^2), D = 4 a c T^3 / (3 kappa rho^2 c_v) */
int orc_parabolic_dt(const orc_cfg *c, const orc_opacity *op, const double *rho,
                     const double *T, double *dtp);
/* number of RKL2 stages for a step dt_h: max(1 + floor((sqrt(9 + 16 dt_h/dt_p) - 1)/2), 3) */
int orc_rkl2_nsts(double dt_h, double dt_p);
/* RKL2 coefficients (mu, nu, mu~, gamma~) of stage j of s */
void orc_rkl2_coeffs(int s, int j, double *mu, double *nu, double *mut, double *gamt);
/* One RKL2 step of thermal diffusion over dt with nsts stages (mode
   ORC_DIFF_*); updates E in U and T (in: guess, out: new temperature). */
int orc_diffuse(const orc_cfg *c, const orc_opacity *op, double *U, const double *Bx,
                const double *By, const double *Bz, double *T, double dt, int nsts,
                int mode);

#ifdef __cplusplus
}
#endif
#endif
