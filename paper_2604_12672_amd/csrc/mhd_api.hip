// mhd_api.hip -- host side of the C ABI declared in include/mhd.h:
// argument validation, device buffers, stage sequencing and error latching.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mhd_internal.h"

struct mhd_ctx {
  mhd::Ctx c;
};

namespace {

thread_local std::string g_init_err;

int fail(mhd_ctx *h, int code, const std::string &msg) {
  if (h) h->c.err = msg;
  return code;
}

int hip_fail(mhd_ctx *h, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, MHD_ERR_HIP, m);
}

#define HIPCHK(h, call)                                      \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call);   \
  } while (0)

// SSP-RK stage coefficients (Sect. 2.9): U_new = a U^n + b U^(s) - c dt R(U^(s))
const double kRK2[2][3] = {{0.0, 1.0, 1.0}, {0.5, 0.5, 0.5}};
const double kRK3[3][3] = {{0.0, 1.0, 1.0}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};

int check_desc(const mhd_grid_desc *d, std::string &msg) {
  if (!d) {
    msg = "descriptor is NULL";
    return MHD_ERR_ARG;
  }
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) {
    msg = "nx, ny, nz must be >= 1";
    return MHD_ERR_ARG;
  }
  if ((double)d->nx * d->ny * (d->nz + 1.0) >= 4294967296.0) {
    msg = "grid too large: nx ny (nz+1) must stay below 2^32 cells";
    return MHD_ERR_ARG;
  }
  // the stage kernel addresses a column within a plane by a 32-bit byte
  // offset: one plane of one field stays below 4 GiB
  if ((double)d->nx * d->ny >= 536870912.0) {
    msg = "grid too large: nx ny must stay below 2^29 cells (one plane below 4 GiB)";
    return MHD_ERR_ARG;
  }
  const double cells = (double)d->nx * d->ny * d->nz;
  if (cells > 4.0e9) {
    msg = "grid too large";
    return MHD_ERR_ARG;
  }
  for (int a = 0; a < 3; ++a)
    if (!(d->hi[a] > d->lo[a]) || !std::isfinite(d->hi[a] - d->lo[a])) {
      msg = "box must have hi > lo on every axis";
      return MHD_ERR_ARG;
    }
  if (d->bc[0] != MHD_BC_PERIODIC || d->bc[1] != MHD_BC_PERIODIC) {
    msg = "x and y boundaries must be periodic";
    return MHD_ERR_ARG;
  }
  if (d->bc[2] != MHD_BC_PERIODIC && d->bc[2] != MHD_BC_REFLECT) {
    msg = "z boundary must be periodic or reflecting";
    return MHD_ERR_ARG;
  }
  if (d->bc[2] == MHD_BC_REFLECT && d->nz < 2) {
    msg = "reflecting z needs nz >= 2";
    return MHD_ERR_ARG;
  }
  if (d->eos != MHD_EOS_IDEAL && d->eos != MHD_EOS_GASRAD) {
    msg = "unknown eos";
    return MHD_ERR_ARG;
  }
  if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) {
    msg = "gamma must be > 1";
    return MHD_ERR_ARG;
  }
  if (d->eos == MHD_EOS_GASRAD) {
    if (!(d->mu > 0.0) || !(d->rgas > 0.0) || !(d->arad >= 0.0)) {
      msg = "gas+radiation EOS needs mu > 0, rgas > 0, arad >= 0";
      return MHD_ERR_ARG;
    }
    if (!(d->newton_tol > 0.0) || d->newton_maxit < 0) {
      msg = "newton_tol must be > 0 and newton_maxit >= 0";
      return MHD_ERR_ARG;
    }
  }
  if (d->grav[0] != 0.0 || d->grav[1] != 0.0 || !std::isfinite(d->grav[2])) {
    msg = "only a finite grav[2] may be nonzero";
    return MHD_ERR_ARG;
  }
  if (d->rk_order != 2 && d->rk_order != 3) {
    msg = "rk_order must be 2 or 3";
    return MHD_ERR_ARG;
  }
  if (d->precision != MHD_PREC_FP64 && d->precision != MHD_PREC_SPLIT) {
    msg = "unknown precision";
    return MHD_ERR_ARG;
  }
  if (d->recon != MHD_RECON_VANLEER && d->recon != MHD_RECON_PPH) {
    msg = "recon must be MHD_RECON_VANLEER or MHD_RECON_PPH";
    return MHD_ERR_ARG;
  }
  if (d->nspecies < 0 || d->nspecies > MHD_MAX_SPECIES) {
    msg = "nspecies must be 0 .. MHD_MAX_SPECIES";
    return MHD_ERR_ARG;
  }
  if (d->flatten != 0 && d->flatten != 1) {
    msg = "flatten must be 0 or 1";
    return MHD_ERR_ARG;
  }
  if (d->flatten && !(d->eps_sf > 0.0 && std::isfinite(d->eps_sf))) {
    msg = "eps_sf must be finite and > 0";
    return MHD_ERR_ARG;
  }
  if (d->eos_guess != MHD_GUESS_PREV_T && d->eos_guess != MHD_GUESS_MLP) {
    msg = "unknown eos_guess";
    return MHD_ERR_ARG;
  }
  if (d->eos_guess == MHD_GUESS_MLP && d->eos != MHD_EOS_GASRAD) {
    msg = "the learned guess needs the gas+radiation EOS";
    return MHD_ERR_ARG;
  }
  if (d->xi_mode < MHD_XI_LINEAR || d->xi_mode > MHD_XI_OFF) {
    msg = "unknown xi_mode";
    return MHD_ERR_ARG;
  }
  if (d->xi_mode != MHD_XI_OFF && !(d->mach_cut > 0.0)) {
    msg = "mach_cut must be > 0";
    return MHD_ERR_ARG;
  }
  return MHD_OK;
}

hipMemcpyKind kind_in(int32_t where) {
  return where == MHD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_out(int32_t where) {
  return where == MHD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

int latched(mhd_ctx *h) {
  mhd::Ctx &c = h->c;
  int flags = 0;
  HIPCHK(h, hipMemcpyAsync(&flags, c.flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(h, hipStreamSynchronize(c.stream));
  if (flags & 2) return fail(h, MHD_ERR_EOS, "temperature inversion failed on the device");
  if (flags & 1)
    return fail(h, MHD_ERR_UNPHYSICAL, "non-physical state on the device (rho <= 0 or e_int <= 0)");
  return MHD_OK;
}

}  // namespace

namespace mhd {
// grid and physics constants of the kernels from a validated descriptor
void fill_phys(const mhd_grid_desc *desc, Phys &ph) {
  ph.nx = desc->nx;
  ph.ny = desc->ny;
  ph.nz = desc->nz;
  ph.reflect = desc->bc[2] == MHD_BC_REFLECT;
  ph.nzf = ph.reflect ? desc->nz + 1 : desc->nz;
  ph.gasrad = desc->eos == MHD_EOS_GASRAD;
  ph.dx = (desc->hi[0] - desc->lo[0]) / desc->nx;
  ph.dy = (desc->hi[1] - desc->lo[1]) / desc->ny;
  ph.dz = (desc->hi[2] - desc->lo[2]) / desc->nz;
  ph.idx = 1.0 / ph.dx;
  ph.idy = 1.0 / ph.dy;
  ph.idz = 1.0 / ph.dz;
  ph.gamma = desc->gamma;
  ph.gm1 = desc->gamma - 1.0;
  ph.igm1 = 1.0 / (desc->gamma - 1.0);
  ph.rmu = ph.gasrad ? desc->rgas / desc->mu : 0.0;
  ph.arad = ph.gasrad ? desc->arad : 0.0;
  ph.cg = ph.gasrad ? desc->rgas / ((desc->gamma - 1.0) * desc->mu) : 0.0;
  ph.icg = ph.cg > 0.0 ? 1.0 / ph.cg : 0.0;
  ph.gz = desc->grav[2];
  ph.newton_tol = desc->newton_tol;
  ph.newton_maxit = desc->newton_maxit;
  ph.xi_mode = desc->xi_mode;
  ph.recon = desc->recon;
  ph.mach_cut = desc->mach_cut;
  ph.imach_cut = desc->mach_cut > 0.0 ? 1.0 / desc->mach_cut : 0.0;
  ph.dims_active[0] = desc->nx > 1;
  ph.dims_active[1] = desc->ny > 1;
  ph.dims_active[2] = desc->nz > 1;
  // after the learned guess Newton gets 8 steps before the bracketed solve
  ph.newton_maxit_mlp = desc->newton_maxit < 8 ? desc->newton_maxit : 8;
}

int validate_desc(const mhd_grid_desc *desc, std::string &msg) { return check_desc(desc, msg); }

// message of a failed call without a context (mhd_last_error(NULL))
void set_context_free_error(const std::string &msg) { g_init_err = msg; }
}  // namespace mhd

namespace mhd {
// accuracy check of the device reciprocal / square root (mhd_mathcheck.hip)
hipError_t launch_math_check(hipStream_t s, const double *x, double *out, long long n);
}  // namespace mhd

extern "C" {

int mhd_init_grid(const mhd_grid_desc *desc, void *hip_stream, mhd_ctx **out) {
  if (!out) return MHD_ERR_ARG;
  *out = nullptr;
  std::string msg;
  int rc = check_desc(desc, msg);
  if (rc) {
    g_init_err = msg;
    return rc;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    g_init_err = "no HIP device";
    return MHD_ERR_NO_DEVICE;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_init_err = std::string("device is not gfx950: ") + prop.gcnArchName;
    return MHD_ERR_NO_DEVICE;
  }
  mhd_ctx *h = new (std::nothrow) mhd_ctx();
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  c.d = *desc;
  c.device = dev;
  c.stream = (hipStream_t)hip_stream;
  mhd::Phys &ph = c.ph;
  mhd::fill_phys(desc, ph);
  c.ncell = (size_t)desc->nx * desc->ny * desc->nz;
  c.nfz = (size_t)desc->nx * desc->ny * ph.nzf;
  // z planes per stage block: a longer segment re-reads fewer halo planes
  // (4 extra per segment), a shorter one gives more blocks.  The blocks run
  // in rounds of (CUs x resident blocks per CU); pick the segment that
  // minimises rounds x (planes + 4) over 16..48 planes.  MHD_ZSEG
  // overrides the choice for tuning.
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    const long long slots = (long long)cus * mhd::stage_blocks_per_cu(c);
    const long long tiles = (long long)((desc->nx + mhd::TB - 1) / mhd::TB) *
                            ((desc->ny + mhd::TB - 1) / mhd::TB);
    const int nz = desc->nz;
    c.zseg = nz < 16 ? nz : 16;
    long long best = -1;
    for (int zs = 16; zs <= 48 && zs <= nz; ++zs) {
      const int segs = (nz + zs - 1) / zs;
      const int len = (nz + segs - 1) / segs;  // balanced segments
      const long long rounds = (tiles * segs + slots - 1) / slots;
      const long long cost = rounds * (len + 4);
      if (best < 0 || cost < best) {
        best = cost;
        c.zseg = len;
      }
    }
  }
  if (const char *zs = std::getenv("MHD_ZSEG")) {
    const int v = std::atoi(zs);
    if (v >= 1 && v <= mhd::ZSEG_MAX) c.zseg = v;
  }
  if (c.zseg > desc->nz) c.zseg = desc->nz;

  auto cleanup = [&](hipError_t e, const char *what) {
    g_init_err = std::string(what) + ": " + hipGetErrorString(e);
    mhd_destroy(h);
    return MHD_ERR_HIP;
  };
  hipError_t e;
  // the allocation-free entry point's scratch address on this device
  if ((e = mhd::noalloc_setup(dev)) != hipSuccess)
    return cleanup(e, "hipGetSymbolAddress scratch");
  for (int s = 0; s < 3; ++s) {
    if ((e = hipMalloc(&c.U[s], sizeof(double) * 5 * c.ncell)) != hipSuccess)
      return cleanup(e, "hipMalloc U");
    if ((e = hipMalloc(&c.Bx[s], sizeof(double) * c.ncell)) != hipSuccess)
      return cleanup(e, "hipMalloc Bx");
    if ((e = hipMalloc(&c.By[s], sizeof(double) * c.ncell)) != hipSuccess)
      return cleanup(e, "hipMalloc By");
    if ((e = hipMalloc(&c.Bz[s], sizeof(double) * c.nfz)) != hipSuccess)
      return cleanup(e, "hipMalloc Bz");
    // the stage kernels never write the wall planes of a reflecting z:
    // every rotating face buffer starts at zero
    if ((e = hipMemsetAsync(c.Bz[s], 0, sizeof(double) * c.nfz, c.stream)) != hipSuccess)
      return cleanup(e, "hipMemset Bz");
  }
  if (desc->eos_guess == MHD_GUESS_MLP)
    if ((e = hipMalloc(&c.mlp, mhd::mlp_bytes())) != hipSuccess) return cleanup(e, "hipMalloc mlp");
  if (ph.gasrad)
    for (int s = 0; s < 2; ++s)
      if ((e = hipMalloc(&c.T[s], sizeof(double) * c.ncell)) != hipSuccess)
        return cleanup(e, "hipMalloc T");
  if ((e = hipMalloc(&c.bg_cc, sizeof(double) * 4 * ph.nz)) != hipSuccess)
    return cleanup(e, "hipMalloc bg");
  if ((e = hipMalloc(&c.bg_fz, sizeof(double) * 4 * ph.nzf)) != hipSuccess)
    return cleanup(e, "hipMalloc bg");
  if ((e = hipMemsetAsync(c.bg_cc, 0, sizeof(double) * 4 * ph.nz, c.stream)) != hipSuccess)
    return cleanup(e, "hipMemset bg");
  if ((e = hipMemsetAsync(c.bg_fz, 0, sizeof(double) * 4 * ph.nzf, c.stream)) != hipSuccess)
    return cleanup(e, "hipMemset bg");
  c.red_len = 16384;
  if ((e = hipMalloc(&c.red, sizeof(double) * c.red_len)) != hipSuccess)
    return cleanup(e, "hipMalloc red");
  if ((e = hipMalloc(&c.dt_dev, sizeof(double))) != hipSuccess)
    return cleanup(e, "hipMalloc dt");
  if ((e = hipMalloc(&c.flags, sizeof(int))) != hipSuccess) return cleanup(e, "hipMalloc flags");
  if ((e = hipMalloc(&c.nstats, sizeof(unsigned long long) * 3)) != hipSuccess)
    return cleanup(e, "hipMalloc stats");
  if (desc->nspecies > 0) {
    for (int s = 0; s < 3; ++s)
      if ((e = hipMalloc(&c.X[s], sizeof(double) * desc->nspecies * c.ncell)) != hipSuccess)
        return cleanup(e, "hipMalloc species");
    for (int a = 0; a < 3; ++a)
      if ((e = hipMalloc(&c.mf[a], sizeof(double) * (a == 2 ? c.nfz : c.ncell))) != hipSuccess)
        return cleanup(e, "hipMalloc mass fluxes");
  }
  if (desc->flatten) {
    if ((e = hipMalloc(&c.shock_p, sizeof(double) * c.ncell)) != hipSuccess)
      return cleanup(e, "hipMalloc shock pressure");
    if ((e = hipMalloc(&c.shock_f, c.ncell)) != hipSuccess)
      return cleanup(e, "hipMalloc shock flags");
  }
  if ((e = hipMemsetAsync(c.flags, 0, sizeof(int), c.stream)) != hipSuccess)
    return cleanup(e, "hipMemset flags");
  if ((e = hipMemsetAsync(c.nstats, 0, sizeof(unsigned long long) * 3, c.stream)) != hipSuccess)
    return cleanup(e, "hipMemset stats");
  if ((e = hipStreamSynchronize(c.stream)) != hipSuccess) return cleanup(e, "sync");
  *out = h;
  return MHD_OK;
}

int mhd_destroy(mhd_ctx *h) {
  if (!h) return MHD_OK;
  mhd::Ctx &c = h->c;
  (void)hipStreamSynchronize(c.stream);
  for (int s = 0; s < 3; ++s) {
    (void)hipFree(c.U[s]);
    (void)hipFree(c.Bx[s]);
    (void)hipFree(c.By[s]);
    (void)hipFree(c.Bz[s]);
  }
  (void)hipFree(c.T[0]);
  (void)hipFree(c.T[1]);
  (void)hipFree(c.bg_cc);
  (void)hipFree(c.bg_fz);
  (void)hipFree(c.heat);
  (void)hipFree(c.fcoef);
  (void)hipFree(c.fzb);
  (void)hipFree(c.red);
  (void)hipFree(c.dt_dev);
  (void)hipFree(c.flags);
  (void)hipFree(c.nstats);
  (void)hipFree(c.mlp);
  (void)hipFree(c.shock_p);
  for (int s = 0; s < 3; ++s) {
    (void)hipFree(c.X[s]);
    (void)hipFree(c.mf[s]);
  }
  (void)hipFree(c.shock_f);
  mhd::DiffBufs &d = c.diff;
  (void)hipFree(d.e0);
  for (int i = 0; i < 3; ++i) (void)hipFree(d.y[i]);
  for (int i = 0; i < 2; ++i) {
    (void)hipFree(d.T[i]);
    (void)hipFree(d.chi[i]);
  }
  (void)hipFree(d.M0);
  (void)hipFree(d.cv0);
  delete h;
  return MHD_OK;
}

const char *mhd_last_error(const mhd_ctx *h) {
  if (!h) return g_init_err.c_str();
  return h->c.err.c_str();
}

int mhd_set_background(mhd_ctx *h, const double *w_cc, const double *w_fz) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!w_cc || !w_fz) return fail(h, MHD_ERR_ARG, "background arrays must not be NULL");
  const int nz = c.ph.nz, nzf = c.ph.nzf;
  for (int f = 0; f < 4; ++f) {
    for (int k = 0; k < nz; ++k)
      if (!std::isfinite(w_cc[f * nz + k])) return fail(h, MHD_ERR_ARG, "background not finite");
    for (int k = 0; k < nzf; ++k)
      if (!std::isfinite(w_fz[f * nzf + k])) return fail(h, MHD_ERR_ARG, "background not finite");
  }
  HIPCHK(h, hipMemcpyAsync(c.bg_cc, w_cc, sizeof(double) * 4 * nz, hipMemcpyHostToDevice, c.stream));
  HIPCHK(h, hipMemcpyAsync(c.bg_fz, w_fz, sizeof(double) * 4 * nzf, hipMemcpyHostToDevice, c.stream));
  HIPCHK(h, hipStreamSynchronize(c.stream));
  return MHD_OK;
}

int mhd_set_sources(mhd_ctx *h, const double *heat, const double *fmodes, int32_t nmodes) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (nmodes < 0 || nmodes > MHD_MAX_FMODES || (nmodes > 0 && !fmodes))
    return fail(h, MHD_ERR_ARG, "nmodes must be 0 .. MHD_MAX_FMODES with a mode array");
  for (int m = 0; m < nmodes; ++m) {
    const double *md = fmodes + 7 * m;
    for (int a = 0; a < 3; ++a)
      if (!(md[a] == std::floor(md[a]) && std::fabs(md[a]) <= (a == 2 ? 2.0 : 4096.0)))
        return fail(h, MHD_ERR_ARG,
                    "mode wavenumbers must be integers, |k_x|, |k_y| <= 4096, |k_z| <= 2");
    for (int a = 3; a < 7; ++a)
      if (!std::isfinite(md[a])) return fail(h, MHD_ERR_ARG, "mode amplitudes and phases must be finite");
  }
  if (heat) {
    for (int k = 0; k < c.ph.nz; ++k)
      if (!std::isfinite(heat[k])) return fail(h, MHD_ERR_ARG, "heating must be finite");
    if (!c.heat) HIPCHK(h, hipMalloc(&c.heat, sizeof(double) * c.ph.nz));
    HIPCHK(h, hipMemcpyAsync(c.heat, heat, sizeof(double) * c.ph.nz, hipMemcpyHostToDevice, c.stream));
  } else if (c.heat) {
    HIPCHK(h, hipStreamSynchronize(c.stream));
    (void)hipFree(c.heat);
    c.heat = nullptr;
  }
  if (nmodes > 0) {
    // f(x) = sum_m a_m cos(alpha_m(x, y) + 2 pi k_z,m Z), alpha_m = 2 pi
    // (k_x X + k_y Y) + phi_m, X = (x - lo)/L at cell centres.  With
    // cos(alpha + beta) = cos alpha cos beta - sin alpha sin beta, each
    // column's forcing is a combination of the z basis {1, cos 2piZ,
    // sin 2piZ, cos 4piZ, sin 4piZ}; its 15 coefficients (3 components x 5)
    // are summed here once, the stage kernel evaluates the combination.
    const int nx = c.ph.nx, ny = c.ph.ny, nz = c.ph.nz;
    const double pi2 = 6.283185307179586476925286766559;
    const size_t nxy = (size_t)nx * ny;
    std::vector<double> coef((size_t)3 * mhd::FZB * nxy, 0.0), zb((size_t)mhd::FZB * nz);
    // cos and sin of alpha = a_x + a_y with a_x = 2 pi k_x X + phi and
    // a_y = 2 pi k_y Y from per-axis tables (angle addition), so a mode
    // costs nx + ny sine/cosine pairs instead of nx ny
    std::vector<double> cx(nx), sx(nx), cy(ny), sy(ny);
    for (int m = 0; m < nmodes; ++m) {
      const double *md = fmodes + 7 * m;
      const int kz = (int)md[2];
      const int d = kz == 0 ? 0 : (kz == 1 || kz == -1 ? 1 : 3);
      const double sg = kz < 0 ? -1.0 : 1.0;
      for (int i = 0; i < nx; ++i) {
        const double ax = pi2 * md[0] * ((i + 0.5) / nx) + md[6];
        cx[i] = std::cos(ax);
        sx[i] = std::sin(ax);
      }
      for (int j = 0; j < ny; ++j) {
        const double ay = pi2 * md[1] * ((j + 0.5) / ny);
        cy[j] = std::cos(ay);
        sy[j] = std::sin(ay);
      }
      for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
          const double ca = cx[i] * cy[j] - sx[i] * sy[j];
          const double sa = sx[i] * cy[j] + cx[i] * sy[j];
          const size_t q = (size_t)j * nx + i;
          for (int cc = 0; cc < 3; ++cc) {
            double *cf = coef.data() + (size_t)(cc * mhd::FZB) * nxy + q;
            cf[(size_t)d * nxy] += md[3 + cc] * ca;
            if (kz != 0) cf[(size_t)(d + 1) * nxy] -= sg * md[3 + cc] * sa;
          }
        }
      }
    }
    for (int k = 0; k < nz; ++k) {
      const double Z = (k + 0.5) / nz;
      zb[k] = 1.0;
      zb[(size_t)nz + k] = std::cos(pi2 * Z);
      zb[(size_t)2 * nz + k] = std::sin(pi2 * Z);
      zb[(size_t)3 * nz + k] = std::cos(2.0 * pi2 * Z);
      zb[(size_t)4 * nz + k] = std::sin(2.0 * pi2 * Z);
    }
    if (!c.fcoef) HIPCHK(h, hipMalloc(&c.fcoef, sizeof(double) * coef.size()));
    if (!c.fzb) HIPCHK(h, hipMalloc(&c.fzb, sizeof(double) * zb.size()));
    HIPCHK(h, hipMemcpyAsync(c.fcoef, coef.data(), sizeof(double) * coef.size(),
                             hipMemcpyHostToDevice, c.stream));
    HIPCHK(h, hipMemcpyAsync(c.fzb, zb.data(), sizeof(double) * zb.size(), hipMemcpyHostToDevice,
                             c.stream));
    HIPCHK(h, hipStreamSynchronize(c.stream));  // the host tables go out of scope
  } else if (c.fcoef) {
    HIPCHK(h, hipStreamSynchronize(c.stream));
    (void)hipFree(c.fcoef);
    (void)hipFree(c.fzb);
    c.fcoef = c.fzb = nullptr;
  }
  HIPCHK(h, hipStreamSynchronize(c.stream));
  return MHD_OK;
}

int mhd_set_state(mhd_ctx *h, const double *U, const double *Bx, const double *By,
                  const double *Bz, const double *T, int32_t where) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!U || !Bx || !By || !Bz) return fail(h, MHD_ERR_ARG, "state arrays must not be NULL");
  if (where != MHD_HOST && where != MHD_DEVICE) return fail(h, MHD_ERR_ARG, "bad `where`");
  const int s = c.cur;
  HIPCHK(h, hipMemcpyAsync(c.U[s], U, sizeof(double) * 5 * c.ncell, kind_in(where), c.stream));
  HIPCHK(h, hipMemcpyAsync(c.Bx[s], Bx, sizeof(double) * c.ncell, kind_in(where), c.stream));
  HIPCHK(h, hipMemcpyAsync(c.By[s], By, sizeof(double) * c.ncell, kind_in(where), c.stream));
  HIPCHK(h, hipMemcpyAsync(c.Bz[s], Bz, sizeof(double) * c.nfz, kind_in(where), c.stream));
  if (c.ph.reflect) HIPCHK(h, mhd::launch_zero_walls(c, c.Bz[s]));
  HIPCHK(h, hipMemsetAsync(c.flags, 0, sizeof(int), c.stream));
  if (c.ph.gasrad && c.d.eos_guess == MHD_GUESS_PREV_T) {
    if (T)
      HIPCHK(h, hipMemcpyAsync(c.T[c.tcur], T, sizeof(double) * c.ncell, kind_in(where), c.stream));
    else
      HIPCHK(h, mhd::launch_init_temperature(c, c.U[s], c.Bx[s], c.By[s], c.Bz[s], nullptr,
                                             c.T[c.tcur]));
  }
  c.have_state = true;
  c.t0_current = false;
  c.p_current = false;
  c.have_species = false;
  return latched(h);
}

int mhd_set_species(mhd_ctx *h, const double *rhoX, int32_t where) {
  if (!h || !rhoX) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (c.d.nspecies <= 0) return fail(h, MHD_ERR_STATE, "context created without species");
  if (!c.have_state) return fail(h, MHD_ERR_STATE, "mhd_set_species before mhd_set_state");
  if (where != MHD_HOST && where != MHD_DEVICE) return fail(h, MHD_ERR_ARG, "bad `where`");
  HIPCHK(h, hipMemcpyAsync(c.X[c.cur], rhoX, sizeof(double) * c.d.nspecies * c.ncell,
                           kind_in(where), c.stream));
  c.have_species = true;
  return latched(h);
}

int mhd_get_species(mhd_ctx *h, double *rhoX, int32_t where) {
  if (!h || !rhoX) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (c.d.nspecies <= 0) return fail(h, MHD_ERR_STATE, "context created without species");
  if (!c.have_species) return fail(h, MHD_ERR_STATE, "mhd_get_species before mhd_set_species");
  if (where != MHD_HOST && where != MHD_DEVICE) return fail(h, MHD_ERR_ARG, "bad `where`");
  HIPCHK(h, hipMemcpyAsync(rhoX, c.X[c.cur], sizeof(double) * c.d.nspecies * c.ncell,
                           kind_out(where), c.stream));
  return latched(h);
}

// The CFL kernel of the current state; with the gas+radiation EOS it also
// stores the converged temperatures where the first stage looks for its
// guess (the previous-T array, or the learned guess array, which then needs
// no guess kernel for that stage), and with flattening the pressure the
// first stage's detector needs.
static hipError_t launch_cfl(mhd::Ctx &c, double cfl) {
  const int n = c.cur;
  const bool learned = c.ph.gasrad && c.d.eos_guess == MHD_GUESS_MLP;
  double *Tout = c.ph.gasrad ? (learned ? c.T[0] : c.T[c.tcur]) : nullptr;
  hipError_t e = mhd::launch_signal_speed(c, c.U[n], c.Bx[n], c.By[n], c.Bz[n],
                                          c.ph.gasrad ? c.T[c.tcur] : nullptr, cfl, c.dt_dev,
                                          Tout, c.d.flatten ? c.shock_p : nullptr);
  if (e == hipSuccess) {
    c.t0_current = learned;
    c.p_current = c.d.flatten != 0;
  }
  return e;
}

static int run_step(mhd_ctx *h, double dt_host, const double *dt_dev) {
  mhd::Ctx &c = h->c;
  if (c.d.eos_guess == MHD_GUESS_MLP && !c.have_mlp)
    return fail(h, MHD_ERR_STATE, "learned guess selected but mhd_set_eos_mlp not called");
  if (c.d.nspecies > 0 && !c.have_species)
    return fail(h, MHD_ERR_STATE, "species context stepped before mhd_set_species");
  const int ns = c.d.rk_order == 3 ? 3 : 2;
  const double(*co)[3] = c.d.rk_order == 3 ? kRK3 : kRK2;
  const int n = c.cur;
  const int a = (n + 1) % 3, b = (n + 2) % 3;
  // stage outputs: RK2 n -> a -> b; RK3 n -> a -> b -> a
  const int outs[3] = {a, b, a};
  int in = n;
  if (c.ph.gasrad)
    HIPCHK(h, hipMemsetAsync(c.nstats, 0, sizeof(unsigned long long) * 3, c.stream));
  for (int s = 0; s < ns; ++s) {
    const int o = outs[s];
    mhd::StagePtrs p;
    p.Us = c.U[in];
    p.Bxs = c.Bx[in];
    p.Bys = c.By[in];
    p.Bzs = c.Bz[in];
    p.U0 = c.U[n];
    p.Bx0 = c.Bx[n];
    p.By0 = c.By[n];
    p.Bz0 = c.Bz[n];
    p.Uo = c.U[o];
    p.Bxo = c.Bx[o];
    p.Byo = c.By[o];
    p.Bzo = c.Bz[o];
    const bool prev_t = c.ph.gasrad && c.d.eos_guess == MHD_GUESS_PREV_T;
    const bool learned = c.ph.gasrad && c.d.eos_guess == MHD_GUESS_MLP;
    const bool reuse = s == 0 && (!learned || c.t0_current) && (!c.d.flatten || c.p_current);
    if (learned && !(reuse && c.t0_current)) {
      // learned guesses of the stage input, polished by FP64 Newton in the
      // guess kernel (with flattening the pressure is taken there too), so
      // the stage starts from converged temperatures; the first stage skips
      // this when the CFL kernel left the converged temperatures of its
      // input
      HIPCHK(h, mhd::launch_mlp_guess(c, p.Us, p.Bxs, p.Bys, p.Bzs, c.T[0],
                                      c.d.flatten ? c.shock_p : nullptr, true, c.nstats));
    }
    p.Tin = prev_t ? c.T[c.tcur] : (learned ? c.T[0] : nullptr);
    p.Tout = prev_t ? c.T[1 - c.tcur] : nullptr;
    p.newton_cap = learned ? c.ph.newton_maxit_mlp : c.ph.newton_maxit;
    if (c.d.flatten) {
      // flags of the stage input, from the same EOS guess the stage uses
      if (!learned && !reuse)
        HIPCHK(h, mhd::launch_shock_pressure(c, p.Us, p.Bxs, p.Bys, p.Bzs, p.Tin, p.newton_cap));
      HIPCHK(h, mhd::launch_shock_flags(c));
      p.flat = c.shock_f;
    }
    p.bg_cc = c.bg_cc;
    p.bg_fz = c.bg_fz;
    p.heat = c.heat;
    p.fcoef = c.fcoef;
    p.fzb = c.fzb;
    p.dt_dev = dt_dev;
    p.flags = c.flags;
    p.newton_stats = c.nstats;
    if (c.d.nspecies > 0) {
      p.mfx = c.mf[0];
      p.mfy = c.mf[1];
      p.mfz = c.mf[2];
    }
    HIPCHK(h, mhd::launch_stage(c, p, co[s][0], co[s][1], co[s][2], dt_host));
    if (c.d.nspecies > 0)
      HIPCHK(h, mhd::launch_species(c, c.U[in], c.X[in], c.X[n], c.X[o], co[s][0], co[s][1],
                                    co[s][2], dt_host, dt_dev, p.flat));
    if (prev_t) c.tcur = 1 - c.tcur;
    in = o;
  }
  c.cur = in;
  c.t0_current = false;
  c.p_current = false;
  return MHD_OK;
}

int mhd_step(mhd_ctx *h, double dt) {
  if (!h) return MHD_ERR_ARG;
  if (!h->c.have_state) return fail(h, MHD_ERR_STATE, "mhd_step before mhd_set_state");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, MHD_ERR_ARG, "dt must be finite and > 0");
  return run_step(h, dt, nullptr);
}

int mhd_advance(mhd_ctx *h, double cfl, int32_t nsteps) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!c.have_state) return fail(h, MHD_ERR_STATE, "mhd_advance before mhd_set_state");
  if (!(cfl > 0.0) || !std::isfinite(cfl) || nsteps < 0)
    return fail(h, MHD_ERR_ARG, "cfl must be > 0 and nsteps >= 0");
  if (c.d.eos_guess == MHD_GUESS_MLP && !c.have_mlp)
    return fail(h, MHD_ERR_STATE, "learned guess selected but mhd_set_eos_mlp not called");
  for (int s = 0; s < nsteps; ++s) {
    HIPCHK(h, launch_cfl(c, cfl));
    int rc = run_step(h, 0.0, c.dt_dev);
    if (rc) return rc;
  }
  return MHD_OK;
}

int mhd_compute_dt(mhd_ctx *h, double cfl, double *dt_out) {
  if (!h || !dt_out) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!c.have_state) return fail(h, MHD_ERR_STATE, "mhd_compute_dt before mhd_set_state");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(h, MHD_ERR_ARG, "cfl must be > 0");
  if (c.d.eos_guess == MHD_GUESS_MLP && !c.have_mlp)
    return fail(h, MHD_ERR_STATE, "learned guess selected but mhd_set_eos_mlp not called");
  HIPCHK(h, launch_cfl(c, cfl));
  double dt = 0.0;
  HIPCHK(h, hipMemcpyAsync(&dt, c.dt_dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  int rc = latched(h);
  if (rc) return rc;
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(h, MHD_ERR_UNPHYSICAL, "signal speed is not finite and positive");
  *dt_out = dt;
  return MHD_OK;
}

int mhd_get_state(mhd_ctx *h, double *U, double *Bx, double *By, double *Bz, double *T,
                  int32_t where) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!c.have_state) return fail(h, MHD_ERR_STATE, "mhd_get_state before mhd_set_state");
  if (where != MHD_HOST && where != MHD_DEVICE) return fail(h, MHD_ERR_ARG, "bad `where`");
  const int s = c.cur;
  if (U) HIPCHK(h, hipMemcpyAsync(U, c.U[s], sizeof(double) * 5 * c.ncell, kind_out(where), c.stream));
  if (Bx) HIPCHK(h, hipMemcpyAsync(Bx, c.Bx[s], sizeof(double) * c.ncell, kind_out(where), c.stream));
  if (By) HIPCHK(h, hipMemcpyAsync(By, c.By[s], sizeof(double) * c.ncell, kind_out(where), c.stream));
  if (Bz) HIPCHK(h, hipMemcpyAsync(Bz, c.Bz[s], sizeof(double) * c.nfz, kind_out(where), c.stream));
  if (T) {
    if (!c.ph.gasrad) return fail(h, MHD_ERR_ARG, "T requested for the ideal-gas EOS");
    // temperature of the current state: Newton from the stored solution of
    // the last stage (previous-T mode, which keeps its guess array), or
    // the bracketed solve (learned mode stores no temperature)
    const bool prev_t = c.d.eos_guess == MHD_GUESS_PREV_T;
    double *dst = prev_t ? c.T[1 - c.tcur] : c.T[0];
    HIPCHK(h, mhd::launch_init_temperature(c, c.U[s], c.Bx[s], c.By[s], c.Bz[s],
                                           prev_t ? c.T[c.tcur] : nullptr, dst));
    HIPCHK(h, hipMemcpyAsync(T, dst, sizeof(double) * c.ncell, kind_out(where), c.stream));
  }
  return latched(h);
}

int mhd_sync(mhd_ctx *h) {
  if (!h) return MHD_ERR_ARG;
  return latched(h);
}

int mhd_shock_flags(mhd_ctx *h, uint8_t *flags, int32_t where) {
  if (!h || !flags) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!c.have_state) return fail(h, MHD_ERR_STATE, "mhd_shock_flags before mhd_set_state");
  if (!c.d.flatten) return fail(h, MHD_ERR_STATE, "context created without shock flattening");
  if (where != MHD_HOST && where != MHD_DEVICE) return fail(h, MHD_ERR_ARG, "bad `where`");
  if (c.d.eos_guess == MHD_GUESS_MLP && !c.have_mlp)
    return fail(h, MHD_ERR_STATE, "learned guess selected but mhd_set_eos_mlp not called");
  const int s = c.cur;
  if (c.ph.gasrad && c.d.eos_guess == MHD_GUESS_MLP)
    HIPCHK(h, mhd::launch_mlp_guess(c, c.U[s], c.Bx[s], c.By[s], c.Bz[s], c.T[0], c.shock_p,
                                    true, nullptr));
  else
    HIPCHK(h, mhd::launch_shock_pressure(c, c.U[s], c.Bx[s], c.By[s], c.Bz[s],
                                         c.ph.gasrad ? c.T[c.tcur] : nullptr, c.ph.newton_maxit));
  HIPCHK(h, mhd::launch_shock_flags(c));
  HIPCHK(h, hipMemcpyAsync(flags, c.shock_f, c.ncell, kind_out(where), c.stream));
  return latched(h);
}

int mhd_diagnostics(mhd_ctx *h, mhd_diag *out) {
  if (!h || !out) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!c.have_state) return fail(h, MHD_ERR_STATE, "mhd_diagnostics before mhd_set_state");
  const int s = c.cur;
  double v[9];
  HIPCHK(h, mhd::launch_diagnostics(c, c.U[s], c.Bx[s], c.By[s], c.Bz[s], v));
  std::memset(out, 0, sizeof(*out));
  out->bface_max = v[2];
  const double bm = v[2] > 0.0 ? v[2] : 1.0;
  out->divb_max = v[0] / bm;
  out->divb_l2 = std::sqrt(v[1] / (double)c.ncell) / bm;
  for (int f = 0; f < 5; ++f) out->total[f] = v[3 + f];
  out->bflux_x0 = v[8];
  unsigned long long st[3] = {0, 0, 0};
  int flags = 0;
  HIPCHK(h, hipMemcpyAsync(st, c.nstats, sizeof(st), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(h, hipMemcpyAsync(&flags, c.flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(h, hipStreamSynchronize(c.stream));
  out->newton_iters = (int64_t)st[0];
  out->newton_max = (int64_t)st[1];
  out->fallbacks = (int64_t)st[2];
  out->error_flags = flags;
  return latched(h);
}

int mhd_set_eos_mlp(mhd_ctx *h, const float *w1, const float *b1, const uint16_t *w2,
                    const float *b2, const uint16_t *w3, float b3, const double *norm) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (c.d.eos_guess != MHD_GUESS_MLP)
    return fail(h, MHD_ERR_STATE, "context was not created with MHD_GUESS_MLP");
  if (!w1 || !b1 || !w2 || !b2 || !w3 || !norm)
    return fail(h, MHD_ERR_ARG, "network arrays must not be NULL");
  auto finite_f = [](const float *a, int n) {
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(a[i])) return false;
    return true;
  };
  if (!finite_f(w1, 128) || !finite_f(b1, 64) || !finite_f(b2, 64) || !std::isfinite(b3))
    return fail(h, MHD_ERR_ARG, "network weights must be finite");
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(norm[i])) return fail(h, MHD_ERR_ARG, "normalisation must be finite");
  if (norm[1] == 0.0 || norm[3] == 0.0 || norm[5] == 0.0)
    return fail(h, MHD_ERR_ARG, "normalisation scales must be nonzero");
  // pack the fragments in the lane order of the kernel (see MlpLds)
  std::vector<unsigned char> buf(mhd::mlp_bytes(), 0);
  auto bf = [](float x) -> uint16_t {  // round to nearest even
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  };
  auto bfv = [](uint16_t b) -> float {
    uint32_t u = (uint32_t)b << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
  };
  uint16_t *a1 = (uint16_t *)buf.data();  // [2][64][4]
  uint16_t *a2 = a1 + 2 * 64 * 4;          // [2][4][64][8]
  float *c2 = (float *)(a2 + 2 * 4 * 64 * 8);  // [2][16][64]
  uint16_t *w3b = (uint16_t *)(c2 + 2 * 16 * 64);  // [64]
  for (int mb = 0; mb < 2; ++mb)
    for (int l = 0; l < 64; ++l) {
      const int m = 32 * mb + (l % 32);
      const float w0 = w1[2 * m], wv1 = w1[2 * m + 1], bb = b1[m];
      const uint16_t w0h = bf(w0), w1h = bf(wv1), bh = bf(bb);
      const uint16_t w0l = bf(w0 - bfv(w0h)), w1l = bf(wv1 - bfv(w1h)), bl = bf(bb - bfv(bh));
      uint16_t *d = a1 + (mb * 64 + l) * 4;
      if (l < 32) {
        d[0] = w0h; d[1] = w0l; d[2] = w0h; d[3] = w1h;
      } else {
        d[0] = w1l; d[1] = w1h; d[2] = bh; d[3] = bl;
      }
      // K block q of the K = 16 layer-2 product: value t of lane l is the
      // hidden unit layer 1 leaves in that lane's register 4(2q + t/4) + t%4
      for (int q = 0; q < 4; ++q)
        for (int t = 0; t < 8; ++t)
          a2[((mb * 4 + q) * 64 + l) * 8 + t] =
              w2[m * 64 + 8 * (2 * q + t / 4) + 4 * (l / 32) + t % 4];
      for (int r = 0; r < 16; ++r)
        c2[(mb * 16 + r) * 64 + l] = b2[32 * mb + 8 * (r / 4) + 4 * (l / 32) + r % 4];
    }
  for (int i = 0; i < 64; ++i) w3b[i] = w3[i];
  HIPCHK(h, hipMemcpyAsync(c.mlp, buf.data(), buf.size(), hipMemcpyHostToDevice, c.stream));
  HIPCHK(h, hipStreamSynchronize(c.stream));
  for (int i = 0; i < 6; ++i) c.ph.mlp_norm[i] = (float)norm[i];
  c.ph.mlp_b3 = b3;
  c.ph.mlp_inv_sT = (float)(1.0 / norm[5]);
  c.have_mlp = true;
  // temperatures and pressures left by a CFL kernel came from the old network
  c.t0_current = false;
  c.p_current = false;
  return MHD_OK;
}

int mhd_eos_solve(mhd_ctx *h, const double *rho, const double *e, const double *T_guess,
                  int64_t n, double *T, double *T0, int64_t stats[3]) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!c.ph.gasrad) return fail(h, MHD_ERR_ARG, "mhd_eos_solve needs the gas+radiation EOS");
  if (!rho || !e || !T || n < 0) return fail(h, MHD_ERR_ARG, "bad arguments");
  if (c.d.eos_guess == MHD_GUESS_MLP && !c.have_mlp)
    return fail(h, MHD_ERR_STATE, "learned guess selected but mhd_set_eos_mlp not called");
  if (n == 0) return MHD_OK;
  if (stats) {
    HIPCHK(h, hipMemsetAsync(c.nstats, 0, sizeof(unsigned long long) * 3, c.stream));
    HIPCHK(h, hipMemsetAsync(c.flags, 0, sizeof(int), c.stream));
  }
  HIPCHK(h, mhd::launch_eos_solve(c, rho, e, c.d.eos_guess == MHD_GUESS_MLP ? nullptr : T_guess,
                                  (long long)n, T, T0, stats != nullptr));
  if (!stats) return MHD_OK;  // asynchronous: errors surface at the next sync
  unsigned long long st[3];
  HIPCHK(h, hipMemcpyAsync(st, c.nstats, sizeof(st), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(h, hipStreamSynchronize(c.stream));
  for (int i = 0; i < 3; ++i) stats[i] = (int64_t)st[i];
  return latched(h);
}

int mhd_set_opacity(mhd_ctx *h, double kappa0, double alpha, double beta, double clight) {
  if (!h) return MHD_ERR_ARG;
  mhd::Ctx &c = h->c;
  if (!c.ph.gasrad) return fail(h, MHD_ERR_ARG, "thermal diffusion needs the gas+radiation EOS");
  if (!(kappa0 > 0.0) || !(clight > 0.0) || !std::isfinite(alpha) || !std::isfinite(beta) ||
      !std::isfinite(kappa0) || !std::isfinite(clight))
    return fail(h, MHD_ERR_ARG, "kappa0 and clight must be finite and > 0");
  c.dparams.pref = 4.0 * c.ph.arad * clight / 3.0;
  c.dparams.alpha = alpha;
  c.dparams.beta = beta;
  c.dparams.ikappa0 = 1.0 / kappa0;
  c.have_opacity = true;
  return MHD_OK;
}

static int diffusion_ready(mhd_ctx *h) {
  mhd::Ctx &c = h->c;
  if (!c.have_state) return fail(h, MHD_ERR_STATE, "diffusion before mhd_set_state");
  if (!c.have_opacity) return fail(h, MHD_ERR_STATE, "mhd_set_opacity not called");
  return MHD_OK;
}

int mhd_parabolic_dt(mhd_ctx *h, double *dtp_out) {
  if (!h || !dtp_out) return MHD_ERR_ARG;
  if (int rc = diffusion_ready(h)) return rc;
  mhd::Ctx &c = h->c;
  const int s = c.cur;
  const double *Tg = c.d.eos_guess == MHD_GUESS_PREV_T ? c.T[c.tcur] : nullptr;
  double *slot = c.red + c.red_len - 1;
  HIPCHK(h, mhd::launch_parabolic_dt(c, c.U[s], c.Bx[s], c.By[s], c.Bz[s], Tg, slot));
  double dtp = 0.0;
  HIPCHK(h, hipMemcpyAsync(&dtp, slot, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  if (int rc = latched(h)) return rc;
  if (!(dtp > 0.0)) return fail(h, MHD_ERR_UNPHYSICAL, "parabolic limit is not positive");
  *dtp_out = dtp;
  return MHD_OK;
}

// RKL2 stage coefficients (Meyer, Balsara & Aslam): b_0 = b_1 = b_2 = 1/3,
// b_j = (j^2 + j - 2) / (2 j (j + 1)); w1 = 4 / (s^2 + s - 2); stage 1:
// mu~ = b_1 w1; stage j >= 2: mu = (2j - 1)/j b_j / b_{j-1},
// nu = -(j - 1)/j b_j / b_{j-2}, mu~ = mu w1, gamma~ = -(1 - b_{j-1}) mu~.
static double rkl2_b(int j) { return j <= 2 ? 1.0 / 3.0 : (j * (double)j + j - 2.0) / (2.0 * j * (j + 1.0)); }

int mhd_diffuse(mhd_ctx *h, double dt, int32_t nsts, int32_t mode, int32_t *nsts_used) {
  if (!h) return MHD_ERR_ARG;
  if (int rc = diffusion_ready(h)) return rc;
  mhd::Ctx &c = h->c;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, MHD_ERR_ARG, "dt must be finite and > 0");
  if (mode != MHD_DIFF_EINT && mode != MHD_DIFF_TEMP) return fail(h, MHD_ERR_ARG, "bad mode");
  if (nsts == 1) return fail(h, MHD_ERR_ARG, "RKL2 needs at least 2 stages");
  if (nsts > 100000) return fail(h, MHD_ERR_ARG, "nsts too large");
  mhd::DiffBufs &d = c.diff;
  if (!d.e0) {
    const size_t bytes = sizeof(double) * c.ncell;
    HIPCHK(h, hipMalloc(&d.e0, bytes));
    for (int i = 0; i < 3; ++i) HIPCHK(h, hipMalloc(&d.y[i], bytes));
    for (int i = 0; i < 2; ++i) {
      HIPCHK(h, hipMalloc(&d.T[i], bytes));
      HIPCHK(h, hipMalloc(&d.chi[i], bytes));
    }
    HIPCHK(h, hipMalloc(&d.M0, bytes));
    HIPCHK(h, hipMalloc(&d.cv0, bytes));
  }
  if (nsts <= 0) {
    double dtp;
    if (int rc = mhd_parabolic_dt(h, &dtp)) return rc;
    const int n = 1 + (int)std::floor(0.5 * (std::sqrt(9.0 + 16.0 * dt / dtp) - 1.0));
    if (n > 100000) return fail(h, MHD_ERR_ARG, "dt needs more than 100000 stages");
    nsts = n > 3 ? n : 3;
  }
  if (nsts_used) *nsts_used = nsts;
  const int s = c.cur;
  const int tform = mode == MHD_DIFF_TEMP;
  const bool prev_t = c.d.eos_guess == MHD_GUESS_PREV_T;
  const double *Tg = prev_t ? c.T[c.tcur] : nullptr;
  HIPCHK(h, mhd::launch_diff_init(c, c.U[s], c.Bx[s], c.By[s], c.Bz[s], Tg));
  // Y_0 is e_int, or T_0 in the temperature form, where the stage values are
  // temperatures themselves and the T buffers only hold T_0
  const double *y0 = tform ? d.T[0] : d.e0;
  const double *p1 = y0, *p2 = y0;
  const double w1 = 4.0 / ((double)nsts * nsts + nsts - 2.0);
  int ta = 0;  // chi (and the e-form temperature) ping-pong between stages
  for (int j = 1; j <= nsts; ++j) {
    double mu = 0.0, nu = 0.0, mut, gamt = 0.0;
    if (j == 1) {
      mut = rkl2_b(1) * w1;
    } else {
      mu = (2.0 * j - 1.0) / j * rkl2_b(j) / rkl2_b(j - 1);
      nu = -(j - 1.0) / j * rkl2_b(j) / rkl2_b(j - 2);
      mut = mu * w1;
      gamt = -(1.0 - rkl2_b(j - 1)) * mut;
    }
    double *out = d.y[(j - 1) % 3];
    const double *Ta = tform ? p1 : d.T[ta];
    double *Tb = tform ? nullptr : d.T[1 - ta];
    HIPCHK(h, mhd::launch_diff_stage(c, c.U[s], Ta, d.chi[ta], y0, p1, p2, out, Tb,
                                     d.chi[1 - ta], tform, j == 1, mu, nu, mut, gamt, dt));
    ta = 1 - ta;
    p2 = p1;
    p1 = out;
  }
  const double *Tlast = tform ? p1 : d.T[ta];
  HIPCHK(h, mhd::launch_diff_finish(c, c.U[s], p1, Tlast, tform, prev_t ? c.T[c.tcur] : nullptr));
  c.t0_current = false;
  c.p_current = false;
  return MHD_OK;
}

int mhd_math_check(const double *x, double *out, int64_t n, void *hip_stream) {
  if (n < 0 || (n > 0 && (!x || !out))) return MHD_ERR_ARG;
  if (n == 0) return MHD_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (mhd::launch_math_check(s, x, out, (long long)n) != hipSuccess) return MHD_ERR_HIP;
  return hipStreamSynchronize(s) == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_launch_info(const mhd_ctx *h, int32_t *tile, int32_t *zseg, int32_t *blocks) {
  if (!h) return MHD_ERR_ARG;
  const mhd::Ctx &c = h->c;
  if (tile) *tile = mhd::TB;
  if (zseg) *zseg = c.zseg;
  if (blocks)
    *blocks = ((c.ph.nx + mhd::TB - 1) / mhd::TB) * ((c.ph.ny + mhd::TB - 1) / mhd::TB) *
              ((c.ph.nz + c.zseg - 1) / c.zseg);
  return MHD_OK;
}

}  // extern "C"
