/*
 * mhd.h -- C ABI of the MI355X (gfx950) explicit finite-volume MHD step.
 *
 * The library advances the ideal-MHD system with gravity and energy /
 * momentum sources (arXiv 2604.12672, Sect. 2.1) by one explicit SSP-RK
 * step (Sect. 2.9) of the well-balanced (Sect. 2.8), van Leer reconstructed
 * (Sect. 2.5), LHLLD (Sect. 2.6), Contact-CT (Sect. 2.4) scheme, with a
 * per-cell Newton inversion T(rho, e_int) for the gas+radiation EOS
 * (Sect. 2.2, eqs. prad/erad).  One fused HIP kernel computes each RK stage;
 * a reduction kernel computes the CFL step (eq. cfl).
 *
 * Grid and storage.  Uniform Cartesian grid of nx*ny*nz cells on the box
 * [lo, hi]; x and y are periodic; z is periodic or reflecting.  All state
 * arrays are FP64, structure-of-arrays, x fastest, interior cells only:
 *   U   [5][nz][ny][nx]  rho, m_x, m_y, m_z, E   (E includes |B_cc|^2 / 2,
 *                        B_cc = mean of the two faces on each axis)
 *   Bx  [nz][ny][nx]     Bx[k][j][i] = B_x on the face x_{i-1/2}
 *   By  [nz][ny][nx]     By[k][j][i] = B_y on the face y_{j-1/2}
 *   Bz  [nzf][ny][nx]    Bz[k][j][i] = B_z on the face z_{k-1/2};
 *                        nzf = nz (periodic z) or nz+1 (reflecting z; the
 *                        wall planes k = 0 and k = nz hold zero)
 *   T   [nz][ny][nx]     temperature (gas+radiation EOS only)
 *
 * Ownership.  The caller owns every pointer it passes; the library copies
 * in and out on its stream and never keeps caller pointers.  The library
 * owns its device buffers (allocated in mhd_init_grid, freed in
 * mhd_destroy).  `where` says whether a pointer is host memory
 * (MHD_HOST) or device memory (MHD_DEVICE, e.g. a torch CUDA tensor).
 *
 * Errors.  Every call returns 0 (MHD_OK) or a negative MHD_ERR_* code and
 * records a message for mhd_last_error.  No exception crosses the ABI.
 * mhd_step / mhd_advance are asynchronous on the context stream; a
 * non-physical state met on the device (rho <= 0, e_int <= 0, EOS failure)
 * is latched in a device flag and returned by the next synchronising call
 * (mhd_compute_dt, mhd_get_state, mhd_diagnostics, mhd_sync).  Calls in the
 * wrong order (e.g. a step before mhd_set_state) return MHD_ERR_STATE.
 * A context is not thread-safe; calls on one context are serialised by the
 * caller.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHD_OK 0
#define MHD_ERR_ARG (-1)        /* invalid argument or unsupported option    */
#define MHD_ERR_NO_DEVICE (-2)  /* no gfx950 device / no HIP runtime         */
#define MHD_ERR_HIP (-3)        /* a HIP runtime call failed                 */
#define MHD_ERR_UNPHYSICAL (-4) /* rho <= 0, e_int <= 0 or non-finite state  */
#define MHD_ERR_EOS (-5)        /* temperature inversion did not converge    */
#define MHD_ERR_STATE (-6)      /* call out of order                         */

#define MHD_BC_PERIODIC 0
#define MHD_BC_REFLECT 1

#define MHD_EOS_IDEAL 0   /* P = (gamma-1) rho e_int                          */
#define MHD_EOS_GASRAD 1  /* P = rho R T/mu + a T^4/3 (eqs. prad, erad)       */

#define MHD_PREC_FP64 0   /* every operation in FP64                          */
#define MHD_PREC_SPLIT 1  /* reconstruction, Riemann flux and EMFs in FP32 on
                             deviations from the background; background, RK
                             accumulation, flux divergence, curl and EOS
                             Newton polish in FP64                             */

#define MHD_GUESS_PREV_T 0 /* Newton starts from the previous solution (Sect. 2.2) */
#define MHD_GUESS_MLP 1    /* Newton starts from the learned guess (mhd_set_eos_mlp) */

#define MHD_XI_LINEAR 0   /* xi = min(1, max(M_L, M_R) / mach_cut)          */
#define MHD_XI_STEP 1     /* xi = max(M_L, M_R) if below mach_cut, else 1   */
#define MHD_XI_OFF 2      /* xi = 1 (plain HLLD)                            */

#define MHD_RECON_VANLEER 0 /* linear, van Leer limited slope (Sect. 2.5)       */
#define MHD_RECON_PPH 1     /* piecewise parabolic: the unlimited parabola of the
                               three-cell stencil (Sect. 2.5, PPH without
                               species)                                        */

#define MHD_DIFF_EINT 0 /* thermal diffusion evolves e_int (EOS every stage)  */
#define MHD_DIFF_TEMP 1 /* evolves T with c_v frozen at the start (Sect. 2.10) */

#define MHD_HOST 0
#define MHD_DEVICE 1

#define MHD_MAX_SPECIES 16

typedef struct mhd_ctx mhd_ctx; /* opaque */

typedef struct {
  int32_t nx, ny, nz;     /* interior cells, each >= 1; nx ny (nz+1) < 2^32,
                             nx ny < 2^29                                      */
  double lo[3], hi[3];    /* box corners, hi > lo                              */
  int32_t bc[3];          /* bc[0] = bc[1] = MHD_BC_PERIODIC;
                             bc[2] = MHD_BC_PERIODIC or MHD_BC_REFLECT        */
  int32_t eos;            /* MHD_EOS_*                                         */
  double gamma;           /* adiabatic index of the gas (> 1)                  */
  double mu, rgas, arad;  /* gas+radiation constants in code units            */
  double grav[3];         /* constant gravity; only grav[2] may be nonzero     */
  int32_t rk_order;       /* 2 (SSP-RK2) or 3 (SSP-RK3)                        */
  int32_t precision;      /* MHD_PREC_*                                        */
  int32_t eos_guess;      /* MHD_GUESS_*                                       */
  double newton_tol;      /* relative residual |de|/e_int (paper: 1e-11)       */
  int32_t newton_maxit;   /* Newton steps before the bracketed solve           */
  double mach_cut;        /* Mach threshold of the LHLLD factor (paper: 0.6)   */
  int32_t xi_mode;        /* MHD_XI_*                                          */
  int32_t recon;          /* MHD_RECON_*                                       */
  int32_t flatten;        /* 1: shock flattening (Sect. 2.7), 0: off           */
  double eps_sf;          /* detector threshold epsilon_SF (paper: 0.2), > 0   */
  int32_t nspecies;       /* passive species 0 .. MHD_MAX_SPECIES (Sect. 2.9)  */
} mhd_grid_desc;

typedef struct {
  double divb_max;        /* max over cells of |div B| dx_min / max |B_face|   */
  double divb_l2;         /* sqrt(mean (div B dx_min)^2) / max |B_face|        */
  double bface_max;       /* max |B_face|                                      */
  double total[5];        /* sums over cells of rho, m_x, m_y, m_z, E          */
  double bflux_x0;        /* sum of Bx over the plane x_{-1/2}                 */
  int64_t newton_iters;   /* Newton steps of the owned cells, summed over the
                             stages of the last step (with the learned guess
                             including the polish in the guess kernel)        */
  int64_t newton_max;     /* largest Newton count of one cell-stage, last step */
  int64_t fallbacks;      /* cell-stages that needed the bracketed solve,
                             last step                                        */
  int32_t error_flags;    /* latched device flags (bit 0 unphysical, bit 1 EOS) */
} mhd_diag;

/* Create a context on the current HIP device, launching on `hip_stream`
   (a hipStream_t; NULL = the null stream).  Validates the descriptor
   (MHD_ERR_ARG), checks for a gfx950 device (MHD_ERR_NO_DEVICE) and
   allocates all device buffers (MHD_ERR_HIP).  On error *out is NULL. */
int mhd_init_grid(const mhd_grid_desc *desc, void *hip_stream, mhd_ctx **out);

/* Hydrostatic background W_hat known a priori (Sect. 2.8, deviation
   method): host arrays w_cc [4][nz] at cell-centre heights and w_fz
   [4][nzf] at z-face heights, rows rho_hat, P_hat, gamma_e_hat,
   gamma_c_hat.  The background has zero velocity and field.  Without this
   call the background is zero (the full state is reconstructed). */
int mhd_set_background(mhd_ctx *ctx, const double *w_cc, const double *w_fz);

/* Most forcing modes of mhd_set_sources. */
#define MHD_MAX_FMODES 4096

/* Energy source per unit volume heat [nz] (host, nullable; the heating and
   cooling layers of the stratified box) and a forcing acceleration given by
   Fourier modes (host, fmodes [nmodes][7], nullable with nmodes = 0; the
   driven-turbulence setup), adding rho f to the momentum and m.f to the
   energy equation (Sect. 2.1 sources); neither is part of the equilibrium
   source S_hat (Sect. 2.8).  Mode m = (k_x, k_y, k_z, a_x, a_y, a_z, phi)
   contributes a cos(2 pi (k_x X + k_y Y + k_z Z) + phi) with
   X = (x - lo[0]) / (hi[0] - lo[0]) (likewise Y, Z) at the cell centre;
   wavenumbers are integers with |k_x|, |k_y| <= 4096 and |k_z| <= 2, at
   most MHD_MAX_FMODES modes (else MHD_ERR_ARG).  The library sums the
   modes once into per-column coefficients of the z basis {1, cos 2piZ,
   sin 2piZ, cos 4piZ, sin 4piZ} (120 B per column) and the stage kernel
   evaluates the forcing of every cell from them (in FP64; the split path
   keeps the coefficients in FP32, 6e-8 of the forcing).  A call replaces
   both sources; synchronises. */
int mhd_set_sources(mhd_ctx *ctx, const double *heat, const double *fmodes,
                    int32_t nmodes);

/* Learned initial guess of the Newton temperature inversion (contexts
   created with MHD_GUESS_MLP; not part of the paper's method).  Network
   2 -> 64 -> 64 -> 1 with ReLU: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
   y = W3 h2 + b3, with x = ((log10 rho - norm[0]) norm[1],
   (log10 e_int - norm[2]) norm[3]) clipped to [-1, 1] and the guess
   T0 = 10^(y / norm[5] + norm[4]).  Host arrays: w1 [64][2] and b1 [64]
   FP32, w2 [64 out][64 in] and w3 [64] BF16 bit patterns, b2 [64] FP32, b3,
   norm [6].  Layers 1 and 2 run on the matrix cores (BF16 operands, FP32
   accumulation), layer 3 as BF16 dot products on the vector unit, in a
   guess kernel that fills the context's guess array from the stage input
   before each stage; the same kernel polishes each guess by FP64 Newton
   (at most 8 steps, then the bracketed solve) and stores the converged
   temperature, which the stage's own Newton iteration starts from.  Must
   precede the first step.  Copies the weights. */
int mhd_set_eos_mlp(mhd_ctx *ctx, const float *w1, const float *b1,
                    const uint16_t *w2, const float *b2, const uint16_t *w3,
                    float b3, const double *norm);

/* Batch temperature inversion on device arrays (gas+radiation only): T[i]
   solves e_int(rho[i], T) = e[i] (Sect. 2.2) from the context's guess mode
   (MHD_GUESS_PREV_T: T_guess[i], or the bracketed solve when T_guess is
   NULL; MHD_GUESS_MLP: the learned guess).  T0 (nullable) receives the
   guess used.  stats (nullable) = {Newton steps, largest count, bracketed
   solves}.  All pointers are device memory.  With stats the call
   synchronises and returns latched device errors; without, it is
   asynchronous on the context stream (errors surface at the next
   synchronising call). */
int mhd_eos_solve(mhd_ctx *ctx, const double *rho, const double *e,
                  const double *T_guess, int64_t n, double *T, double *T0,
                  int64_t stats[3]);

/* Load the state.  T (nullable) is the initial temperature guess for
   MHD_GUESS_PREV_T; when NULL the library solves T with the bracketed
   method.  The wall planes of Bz are forced to zero for a reflecting z. */
int mhd_set_state(mhd_ctx *ctx, const double *U, const double *Bx,
                  const double *By, const double *Bz, const double *T,
                  int32_t where);

/* CFL step dt = cfl / max_cells sum_s (|v_s| + c_f,s)/dx_s (eq. cfl), axes
   with one cell left out.  Synchronises the stream; returns latched device
   errors. */
int mhd_compute_dt(mhd_ctx *ctx, double cfl, double *dt_out);

/* One SSP-RK step of size dt > 0 (asynchronous). */
int mhd_step(mhd_ctx *ctx, double dt);

/* nsteps steps, each with dt = cfl / (max signal speed) computed on the
   device from the state at the start of the step (asynchronous; no host
   round trip).  Equivalent to nsteps x (mhd_compute_dt; mhd_step). */
int mhd_advance(mhd_ctx *ctx, double cfl, int32_t nsteps);

/* Copy the state out (synchronises).  T (nullable) receives the
   temperature of the current state (gas+radiation only), solved on demand;
   the guess kept for the next step is not changed. */
int mhd_get_state(mhd_ctx *ctx, double *U, double *Bx, double *By, double *Bz,
                  double *T, int32_t where);

/* Passive species (Sect. 2.9): rhoX [ns][nz][ny][nx], the partial
   densities rho X_l (FP64, `where` as for mhd_set_state), for contexts
   with nspecies = ns > 0 (else MHD_ERR_STATE).  Each RK stage advects them
   with the stage's face mass fluxes: the mass fractions are reconstructed
   like the primitives (van Leer; in PPH mode a parabola limited to stay
   monotone; van Leer in flattened cells), rescaled on each side of a face
   to sum to one, and taken from the upwind side of the mass flux, so the
   species masses add up to the density.  mhd_set_species must follow
   mhd_set_state before the first step; mhd_get_species synchronises. */
int mhd_set_species(mhd_ctx *ctx, const double *rhoX, int32_t where);
int mhd_get_species(mhd_ctx *ctx, double *rhoX, int32_t where);

/* Shock-flattening flags (Sect. 2.7) of the current state, one byte per
   cell [nz][ny][nx] (1 = flattened: van Leer reconstruction and HLL on its
   faces), as the next stage would compute them: the detector on the thermal
   pressure, dilated over the 5x5x5 neighbourhood.  Contexts created with
   flatten = 1 only (else MHD_ERR_STATE).  Synchronises. */
int mhd_shock_flags(mhd_ctx *ctx, uint8_t *flags, int32_t where);

/* Wait for queued work; returns latched device errors. */
int mhd_sync(mhd_ctx *ctx);

/* div B (eq. divb), conservation totals, Newton statistics (synchronises). */
int mhd_diagnostics(mhd_ctx *ctx, mhd_diag *out);

/* ---- thermal diffusion with RKL2 super-time-stepping (Sect. 2.10) ---- */

/* Opacity law kappa = kappa0 rho^alpha T^beta (a stand-in for the paper's
   tabulated or fitted opacities) and the speed of light in code units;
   the face conductivity is (4 a c / 3) times the harmonic mean of
   chi = T^3 / (kappa rho).  Gas+radiation EOS only; kappa0, clight > 0. */
int mhd_set_opacity(mhd_ctx *ctx, double kappa0, double alpha, double beta,
                    double clight);

/* Parabolic stability limit dt_p = 1 / (2 max sum_s D / dx_s^2),
   D = 4 a c T^3 / (3 kappa rho^2 c_v), of the current state (synchronises). */
int mhd_parabolic_dt(mhd_ctx *ctx, double *dtp_out);

/* One RKL2 step of rho de_int/dt = div(K grad T) over dt (density, velocity
   and field fixed; E changes by rho (e_new - e_old)), with nsts stages
   (2 <= nsts <= 100000, else MHD_ERR_ARG), or when nsts <= 0 the paper's
   count max(1 + floor((sqrt(9 + 16 dt/dt_p) - 1)/2), 3) (that computes dt_p
   and synchronises).  mode MHD_DIFF_*.
   *nsts_used (nullable) receives the stage count.  Reflecting z walls are
   insulating.  Asynchronous otherwise; errors latch as for mhd_step.  The
   work arrays (10 doubles per cell) are allocated on the first call. */
int mhd_diffuse(mhd_ctx *ctx, double dt, int32_t nsts, int32_t mode,
                int32_t *nsts_used);

/* ---- allocation-free CFL step ---- */

/* Device scratch of mhd_compute_dt_noalloc per device (bytes). */
#define MHD_NOALLOC_SCRATCH_BYTES ((2048 + 64) * 8)

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the CFL
   step of mhd_compute_dt, dt = cfl / max_cells sum_s (|v_s| + c_f,s)/dx_s
   (eq. cfl, axes with one cell left out), of a state held in the caller's
   device memory, without a context.
     desc        grid and EOS as for mhd_init_grid (validated the same way);
                 eos_guess must be MHD_GUESS_PREV_T; the scheme options are
                 not used
     U, Bx, By, Bz  device arrays in the layout of mhd_set_state
     T           device temperature guesses of the gas+radiation inversion,
                 or NULL (bracketed solve); ignored for the ideal gas
     dt_out      one device double, receives dt
     flags_out   one device int32 (nullable), receives 0 or the error bits
                 of mhd_diag.error_flags (1 non-physical, 2 EOS failure)
     hip_stream  the stream to run on (NULL: the null stream)
   Asynchronous on hip_stream; allocates nothing and never synchronises.
   The per-block maxima and the error bits live in a fixed device array of
   MHD_NOALLOC_SCRATCH_BYTES on each device, kept until the process ends and
   shared by every call on that device: calls that overlap on one device
   (on different streams or threads) race and must be serialised by the
   caller.  Any grid the descriptor check accepts fits (the reduction
   strides over cells beyond 2048 blocks of 256); larger grids
   (nx ny (nz+1) >= 2^32 or nx ny >= 2^29) and invalid arguments return
   MHD_ERR_ARG, a device other than gfx950 MHD_ERR_NO_DEVICE, a failed
   launch MHD_ERR_HIP, with the message in mhd_last_error(NULL).  The result is bit for bit the
   one mhd_compute_dt gives for the same state and guesses. */
int mhd_compute_dt_noalloc(const mhd_grid_desc *desc, const double *U, const double *Bx,
                           const double *By, const double *Bz, const double *T, double cfl,
                           double *dt_out, int32_t *flags_out, void *hip_stream);

/* Message of the last failed call on this context ("" if none); for
   ctx == NULL, the message of the last failed mhd_init_grid or
   mhd_compute_dt_noalloc on this thread. */
const char *mhd_last_error(const mhd_ctx *ctx);

/* Free the context and its device buffers (NULL is a no-op). */
int mhd_destroy(mhd_ctx *ctx);

/* Kernel launch geometry of the stage kernel (for tests and profiling):
   tile edge in cells and z-segment length in planes. */
int mhd_launch_info(const mhd_ctx *ctx, int32_t *tile, int32_t *zseg,
                    int32_t *blocks);

/* Accuracy check of the device arithmetic (for tests): evaluates, for each
   of the n device doubles x[i] > 0, the reciprocal and square root the
   kernels use, into the device array out of 4 n doubles:
     out[i]       1/x, the EOS / primitive / update reciprocal
                  (refined hardware seed, within half an ulp)
     out[n+i]     1/x, the flux-arithmetic reciprocal (one refinement step)
     out[2n+i]    sqrt(x), the full sequence
     out[3n+i]    sqrt(x), the flux-arithmetic one (one refinement step)
   hip_stream: the stream to run on (NULL: the default stream); the call
   synchronises it.  Returns MHD_ERR_ARG for n < 0 or NULL arrays with
   n > 0, MHD_ERR_HIP if the launch fails. */
int mhd_math_check(const double *x, double *out, int64_t n, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
