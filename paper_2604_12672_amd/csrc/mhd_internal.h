// mhd_internal.h -- shared declarations of the HIP library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/mhd.h"

namespace mhd {

// Stage-kernel tile: 16 x 16 threads, one cell column each; the inner
// 14 x 14 columns are the outputs, the outer ring is the reconstruction
// halo.  The block marches along z over a segment of ZSEG planes.
constexpr int TT = 16;        // threads per tile edge
constexpr int TB = TT - 2;    // output columns per tile edge
constexpr int NTHREADS = TT * TT;
// z basis of the forcing modes: wavenumbers |k_z| <= 2
constexpr int FZB = 5;
// Longest z segment of a stage block (the block stages the background
// profile of its segment and halo in LDS).
constexpr int ZSEG_MAX = 64;

// Physics and grid constants passed by value to every kernel.
struct Phys {
  int nx, ny, nz, nzf;
  int reflect;        // z boundary: 1 = reflecting walls
  int gasrad;         // 1 = gas+radiation EOS
  double dx, dy, dz, idx, idy, idz;
  double gamma, gm1, igm1;
  double rmu, arad, cg;  // R/mu, a, C_g = R/((gamma-1) mu)
  double icg;            // 1 / C_g
  double gz;
  double newton_tol;
  int newton_maxit;
  int xi_mode;
  int recon;  // MHD_RECON_*
  double mach_cut, imach_cut;
  int dims_active[3];  // axis has more than one cell
  int newton_maxit_mlp;  // Newton cap after the learned guess
  float mlp_norm[6];     // c_rho, s_rho, c_e, s_e, c_T, s_T
  float mlp_b3, mlp_inv_sT;
};

// Pointers of one stage launch.
struct StagePtrs {
  const double *Us, *Bxs, *Bys, *Bzs;  // stage input U^(s)
  const double *U0, *Bx0, *By0, *Bz0;  // step base U^(n) (read when a != 0)
  double *Uo, *Bxo, *Byo, *Bzo;        // stage output
  const double *Tin;                   // EOS guess (gas+radiation)
  double *Tout;                        // EOS solution (owned cells)
  const double *bg_cc, *bg_fz;         // [4][nz], [4][nzf]
  const double *heat;                  // nullable
  // forcing from Fourier modes (nullable): per column the coefficients of
  // the z basis {1, cos 2piZ, sin 2piZ, cos 4piZ, sin 4piZ} for each
  // component, fcoef [3 * FZB][ny][nx], and that basis at the cell
  // centres, fzb [FZB][nz]
  const double *fcoef, *fzb;
  const double *dt_dev;                // device dt (nullable: use dt_host)
  int newton_cap;                      // Newton steps before the bracketed solve
  const uint8_t *flat = nullptr;       // shock-flattening flags [n] (nullable)
  double *mfx = nullptr, *mfy = nullptr, *mfz = nullptr;  // face mass fluxes out
                                       // (lower faces; nullable: no species)
  int *flags;                          // latched error flags
  unsigned long long *newton_stats;    // [3]: iterations, max, fallbacks
};

// Thermal diffusion (RKL2): opacity law and conductivity prefactor
struct DiffParams {
  double pref;      // 4 a c / 3 (code units)
  double alpha, beta;
  double ikappa0;   // 1 / kappa0
};

// RKL2 work arrays (allocated on the first mhd_diffuse)
struct DiffBufs {
  double *e0 = nullptr;                 // e_int at the start
  double *y[3] = {nullptr, nullptr, nullptr};  // stage values Y_j, rotated
  double *T[2] = {nullptr, nullptr};    // temperature of the last two stages (T[0]: T_0)
  double *chi[2] = {nullptr, nullptr};  // chi = T^3 / (kappa rho) of the same
  double *M0 = nullptr;                 // M[T_0] (over c_v0 in the T form)
  double *cv0 = nullptr;                // c_v at the start
};

struct Ctx {
  mhd_grid_desc d;
  Phys ph;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t ncell = 0, nfz = 0;
  // three state buffers (rotated): U [5][n], Bx [n], By [n], Bz [nfz]
  double *U[3] = {nullptr, nullptr, nullptr};
  double *Bx[3] = {nullptr, nullptr, nullptr};
  double *By[3] = {nullptr, nullptr, nullptr};
  double *Bz[3] = {nullptr, nullptr, nullptr};
  int cur = 0;  // index of the current state
  double *T[2] = {nullptr, nullptr};
  int tcur = 0;
  double *bg_cc = nullptr, *bg_fz = nullptr;
  double *heat = nullptr;
  double *fcoef = nullptr, *fzb = nullptr;  // forcing tables (see StagePtrs)
  double *dt_dev = nullptr;       // [1]
  void *mlp = nullptr;            // packed guess network on the device
  bool have_mlp = false;
  double *red = nullptr;          // reduction scratch
  size_t red_len = 0;
  int *flags = nullptr;           // [1]
  unsigned long long *nstats = nullptr;  // [3]
  bool have_state = false;
  DiffParams dparams{};
  bool have_opacity = false;
  DiffBufs diff;
  // shock flattening: thermal pressure of the stage input and the flags
  // (one byte per cell), allocated when enabled
  double *shock_p = nullptr;
  uint8_t *shock_f = nullptr;
  // passive species: rho X_l [ns][n] per state buffer (rotated with U) and
  // the face mass fluxes of the current stage (x, y: [n]; z: [nfz])
  double *X[3] = {nullptr, nullptr, nullptr};
  double *mf[3] = {nullptr, nullptr, nullptr};
  bool have_species = false;
  // learned guess: T[0] holds the converged temperature of the current
  // state (left by the CFL kernel), so the first stage needs no guess kernel
  bool t0_current = false;
  // flattening: shock_p holds the pressure of the current state (also left
  // by the CFL kernel), so the first stage needs no pressure pass
  bool p_current = false;
  int zseg = 32;
  std::string err;
};

// launchers (mhd_kernels.hip)
hipError_t launch_stage(const Ctx &c, const StagePtrs &p, double a, double b,
                        double cc, double dt_host);
// the CFL step into dt_dev; with Tout (gas+radiation, nullable) the
// converged temperature of every cell is stored there as well, with Pout
// (nullable) the thermal pressure
hipError_t launch_signal_speed(const Ctx &c, const double *U, const double *Bx,
                               const double *By, const double *Bz,
                               const double *T, double cfl, double *dt_dev,
                               double *Tout = nullptr, double *Pout = nullptr);
// most blocks of the CFL reduction (grid-stride beyond that)
constexpr int CFL_MAX_BLOCKS = 2048;
// the CFL kernels on explicit buffers: per-block partial maxima in
// partial[0 .. cfl_partial_blocks(n)), the largest signal speed into
// smax_out, cfl / smax into dt_dev, error bits ORed into flags; mlp is the
// packed guess network (learned mode only, else NULL)
int cfl_partial_blocks(size_t ncell);
hipError_t launch_signal_speed_raw(const Phys &ph, hipStream_t stream, bool learned,
                                   const double *U, const double *Bx, const double *By,
                                   const double *Bz, const double *T, const void *mlp,
                                   double *partial, int *flags, double cfl, double *dt_dev,
                                   double *smax_out, double *Tout, double *Pout);
// descriptor checks and kernel constants shared by every entry point
int validate_desc(const mhd_grid_desc *desc, std::string &msg);
void fill_phys(const mhd_grid_desc *desc, Phys &ph);
void set_context_free_error(const std::string &msg);
// device address of the allocation-free entry point's scratch array on
// device dev (the current device), resolved once (mhd_noalloc.hip)
hipError_t noalloc_setup(int dev);
hipError_t launch_init_temperature(const Ctx &c, const double *U,
                                   const double *Bx, const double *By,
                                   const double *Bz, const double *Tg, double *T);
hipError_t launch_diagnostics(const Ctx &c, const double *U, const double *Bx,
                              const double *By, const double *Bz,
                              double *out /* host, 12 */);
hipError_t launch_zero_walls(const Ctx &c, double *Bz);
size_t mlp_bytes();
// resident stage blocks per CU for the context's kernel variant (>= 1)
int stage_blocks_per_cu(const Ctx &c);
// learned guesses into Tg; with P (nullable) also Newton-polished there and
// the thermal pressure into P
hipError_t launch_mlp_guess(const Ctx &c, const double *U, const double *Bx, const double *By,
                            const double *Bz, double *Tg, double *P, bool polish,
                            unsigned long long *stats);
hipError_t launch_diff_init(const Ctx &c, const double *U, const double *Bx, const double *By,
                            const double *Bz, const double *Tg);
hipError_t launch_diff_stage(const Ctx &c, const double *U, const double *Ta, const double *chia,
                             const double *y0, const double *y1, const double *y2, double *yn,
                             double *Tb, double *chib, int tform, int first, double mu,
                             double nu, double mut, double gamt, double dt);
hipError_t launch_diff_finish(const Ctx &c, double *U, const double *ylast, const double *Tlast,
                              int tform, double *Tstore);
hipError_t launch_parabolic_dt(const Ctx &c, const double *U, const double *Bx,
                               const double *By, const double *Bz, const double *Tg,
                               double *dtp_dev);
// shock flattening (mhd_flatten.hip): the thermal pressure of a stage input
// into c.shock_p, then the flags from it into c.shock_f
hipError_t launch_shock_pressure(const Ctx &c, const double *U, const double *Bx,
                                 const double *By, const double *Bz, const double *Tg,
                                 int newton_cap);
hipError_t launch_shock_flags(const Ctx &c);
// species update of one RK stage (mhd_species.hip): Xo = a X0 + b Xs -
// c dt div(F_mass X_up); rho is the stage input density
hipError_t launch_species(const Ctx &c, const double *rho, const double *Xs, const double *X0,
                          double *Xo, double a, double b, double cc, double dt_host,
                          const double *dt_dev, const uint8_t *flat);
hipError_t launch_eos_solve(const Ctx &c, const double *rho, const double *e,
                            const double *tguess, long long n, double *T, double *T0,
                            bool stats);

}  // namespace mhd
