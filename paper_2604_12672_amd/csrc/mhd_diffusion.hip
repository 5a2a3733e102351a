// mhd_diffusion.hip -- thermal diffusion with RKL2 super-time-stepping
// (Sect. 2.10) on gfx950.
//
// The operator M[T] = (1/rho) div(K grad T) uses the harmonic mean of
// chi = T^3 / (kappa rho) for the face conductivity K = (4 a c / 3) chi_f
// and a power-law opacity kappa = kappa0 rho^alpha T^beta.  One kernel per
// RKL2 stage: every cell reads T and chi of itself and its six neighbours
// from the previous stage (two ping-pong buffers), forms M, combines the
// stage (mu, nu, mu~, gamma~ of Meyer, Balsara & Aslam), and writes its new
// value together with its new T (Newton from the previous stage's T in the
// internal-energy form; the value itself in the temperature form) and chi,
// so the next stage reads them without recomputing powers.  Memory-bound
// stencil work: coalesced SoA streams, neighbours from the caches.
#include <hip/hip_runtime.h>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {

__device__ __forceinline__ double chi_of(const DiffParams &dp, double rho, double T) {
  // T^3 / (kappa0 rho^alpha T^beta rho) = T^(3 - beta) rho^(-1 - alpha) / kappa0
  return exp((3.0 - dp.beta) * log(T) - (1.0 + dp.alpha) * log(rho)) * dp.ikappa0;
}

// M[T] at cell q (times 1/c_v0 in the temperature form is left to the caller)
__device__ __forceinline__ double diff_rhs(const Phys &ph, const DiffParams &dp,
                                           const double *__restrict__ rho,
                                           const double *__restrict__ T,
                                           const double *__restrict__ chi, size_t q, int i,
                                           int j, int k) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const double tq = T[q], cq = chi[q];
  double div = 0.0;
  // lower and upper neighbour offsets per active axis
  auto face = [&](size_t qn, double inv_dx) {
    // flux from q to its neighbour: -K (T_n - T_q) / dx; its divergence
    // contribution to q is -(flux out) / dx
    const double cn = chi[qn];
    const double K = dp.pref * 2.0 * cq * cn * rcp<double>(cq + cn);
    return K * (T[qn] - tq) * inv_dx * inv_dx;
  };
  if (ph.dims_active[0]) {
    const int im = i == 0 ? ph.nx - 1 : i - 1, ip = i + 1 == ph.nx ? 0 : i + 1;
    div += face(q - i + im, ph.idx) + face(q - i + ip, ph.idx);
  }
  if (ph.dims_active[1]) {
    const int jm = j == 0 ? ph.ny - 1 : j - 1, jp = j + 1 == ph.ny ? 0 : j + 1;
    div += face(q + (size_t)(jm - j) * ph.nx, ph.idy) + face(q + (size_t)(jp - j) * ph.nx, ph.idy);
  }
  if (ph.dims_active[2]) {
    // a reflecting wall is insulating: no flux through it
    if (!(ph.reflect && k == 0)) {
      const int km = k == 0 ? ph.nz - 1 : k - 1;
      div += face(q + ((size_t)km - (size_t)k) * plane, ph.idz);
    }
    if (!(ph.reflect && k + 1 == ph.nz)) {
      const int kp = k + 1 == ph.nz ? 0 : k + 1;
      div += face(q + ((size_t)kp - (size_t)k) * plane, ph.idz);
    }
  }
  return div * rcp<double>(rho[q]);
}

// e_int, T (Newton from Tg, or the bracketed solve), c_v and chi of every
// cell of the state
__global__ __launch_bounds__(256) void diff_init_kernel(
    Phys ph, DiffParams dp, const double *__restrict__ U, const double *__restrict__ Bx,
    const double *__restrict__ By, const double *__restrict__ Bz,
    const double *__restrict__ Tg, double *__restrict__ e0, double *__restrict__ T0,
    double *__restrict__ chi0, double *__restrict__ cv0, int *flags) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  size_t c0, c1;
  block_cells(n, c0, c1);
  for (size_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const int ip = i + 1 == ph.nx ? 0 : i + 1;
    const int jp = j + 1 == ph.ny ? 0 : j + 1;
    const int kp = ph.reflect ? k + 1 : (k + 1 == ph.nz ? 0 : k + 1);
    double u[5], b[3];
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = U[f * n + q];
    b[0] = 0.5 * (Bx[q] + Bx[q - i + ip]);
    b[1] = 0.5 * (By[q] + By[q + (size_t)(jp - j) * ph.nx]);
    b[2] = 0.5 * (Bz[q] + Bz[(size_t)kp * plane + (q - (size_t)k * plane)]);
    const double rho = u[0];
    const double e = specific_eint(u, b);
    double t = NAN;
    int it = 0, fb = 0;
    int bad = (rho > 0.0 && e > 0.0 && e < INFINITY) ? 0 : 1;
    if (!bad && eos_temperature(ph, rho, e, Tg ? Tg[q] : NAN, ph.newton_maxit, t, it, fb))
      bad = 2;
    if (bad) atomicOr(flags, bad);
    const double t3 = t * t * t;
    e0[q] = e;
    T0[q] = t;
    chi0[q] = chi_of(dp, rho, t);
    cv0[q] = ph.cg + 4.0 * ph.arad * t3 * rcp<double>(rho);
  }
}

// One RKL2 stage: yn = mu y1 + nu y2 + (1 - mu - nu) y0 + mut dt M[Ta] +
// gamt dt M0 (first stage: yn = y0 + mut dt M[Ta], and M0 = M[Ta] is kept),
// then the temperature and chi of yn.  In the temperature form (TF) the
// stage value is the temperature: Ta is y1 itself (y0 in the first stage),
// M is divided by c_v0, and no separate temperature is read or written.
template <bool TF>
__global__ __launch_bounds__(256) void diff_stage_kernel(
    Phys ph, DiffParams dp, const double *__restrict__ U, const double *__restrict__ Ta,
    const double *__restrict__ chia, const double *__restrict__ y0,
    const double *__restrict__ y1, const double *__restrict__ y2, double *__restrict__ M0,
    const double *__restrict__ cv0, int first, double mu, double nu, double mut,
    double gamt, double dt, double *__restrict__ yn, double *__restrict__ Tb,
    double *__restrict__ chib, int *flags) {
  const size_t n = (size_t)ph.nx * ph.ny * ph.nz;
  const double *rho = U;
  const double *yp = TF ? Ta : y1;
  size_t c0, c1;
  block_cells(n, c0, c1);
  for (size_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const double r = rho[q];
    double M = diff_rhs(ph, dp, rho, Ta, chia, q, i, j, k);
    if (TF) M *= rcp<double>(cv0[q]);
    double v;
    if (first) {
      M0[q] = M;
      v = y0[q] + mut * dt * M;
    } else {
      v = mu * yp[q] + nu * y2[q] + (1.0 - mu - nu) * y0[q] + mut * dt * M + gamt * dt * M0[q];
    }
    yn[q] = v;
    double t = v;
    if (!TF) {
      int it, fb;
      if (!(v > 0.0) || eos_temperature(ph, r, v, Ta[q], ph.newton_maxit, t, it, fb))
        atomicOr(flags, 2);
      Tb[q] = t;
    } else if (!(v > 0.0)) {
      atomicOr(flags, 2);
    }
    chib[q] = chi_of(dp, r, t);
  }
}

// E += rho (e_new - e0); the final temperature is kept as the next guess
__global__ __launch_bounds__(256) void diff_finish_kernel(
    Phys ph, double *__restrict__ U, const double *__restrict__ e0,
    const double *__restrict__ ylast, const double *__restrict__ Tlast, int tform,
    double *__restrict__ Tstore) {
  const size_t n = (size_t)ph.nx * ph.ny * ph.nz;
  size_t c0, c1;
  block_cells(n, c0, c1);
  for (size_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) {
    const double rho = U[q];
    const double enew = tform ? specific_eint_rt(ph, rho, Tlast[q]) : ylast[q];
    U[4 * n + q] += rho * (enew - e0[q]);
    if (Tstore) Tstore[q] = Tlast[q];
  }
}

// parabolic limit: per-block maxima of sum_s D / dx_s^2, then 0.5 / max
__global__ __launch_bounds__(256) void parabolic_kernel(
    Phys ph, DiffParams dp, const double *__restrict__ U, const double *__restrict__ Bx,
    const double *__restrict__ By, const double *__restrict__ Bz,
    const double *__restrict__ Tg, double *__restrict__ partial, int *flags) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  double m = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const int ip = i + 1 == ph.nx ? 0 : i + 1;
    const int jp = j + 1 == ph.ny ? 0 : j + 1;
    const int kp = ph.reflect ? k + 1 : (k + 1 == ph.nz ? 0 : k + 1);
    double u[5], b[3];
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = U[f * n + q];
    b[0] = 0.5 * (Bx[q] + Bx[q - i + ip]);
    b[1] = 0.5 * (By[q] + By[q + (size_t)(jp - j) * ph.nx]);
    b[2] = 0.5 * (Bz[q] + Bz[(size_t)kp * plane + (q - (size_t)k * plane)]);
    const double rho = u[0], e = specific_eint(u, b);
    double t = NAN;
    int it = 0, fb = 0;
    if (!(rho > 0.0 && e > 0.0) ||
        eos_temperature(ph, rho, e, Tg ? Tg[q] : NAN, ph.newton_maxit, t, it, fb)) {
      atomicOr(flags, 2);
      continue;
    }
    const double t3 = t * t * t;
    const double cv = ph.cg + 4.0 * ph.arad * t3 * rcp<double>(rho);
    // D = (4 a c / 3) T^3 / (kappa rho^2 c_v) = pref chi / (rho c_v)
    const double D = dp.pref * chi_of(dp, rho, t) * rcp<double>(rho * cv);
    double s = 0.0;
    if (ph.dims_active[0]) s += D * ph.idx * ph.idx;
    if (ph.dims_active[1]) s += D * ph.idy * ph.idy;
    if (ph.dims_active[2]) s += D * ph.idz * ph.idz;
    m = s > m ? s : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double m2 = __shfl_xor(m, o);
    m = m2 > m ? m2 : m;
  }
  __shared__ double sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sm[0];
    for (int w = 1; w < 4; ++w) r = sm[w] > r ? sm[w] : r;
    partial[blockIdx.x] = r;
  }
}

__global__ void parabolic_finish_kernel(const double *__restrict__ partial, int nb,
                                        double *dtp) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = partial[i] > m ? partial[i] : m;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && sm[threadIdx.x + s] > sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *dtp = 0.5 / sm[0];
}

static int grid_blocks(const Ctx &c) {
  long long nb = (long long)((c.ncell + 255) / 256);
  return (int)(nb < 65536 ? nb : 65536);
}

hipError_t launch_diff_init(const Ctx &c, const double *U, const double *Bx, const double *By,
                            const double *Bz, const double *Tg) {
  const DiffBufs &d = c.diff;
  hipLaunchKernelGGL(diff_init_kernel, dim3(grid_blocks(c)), dim3(256), 0, c.stream, c.ph,
                     c.dparams, U, Bx, By, Bz, Tg, d.e0, d.T[0], d.chi[0], d.cv0, c.flags);
  return hipGetLastError();
}

hipError_t launch_diff_stage(const Ctx &c, const double *U, const double *Ta, const double *chia,
                             const double *y0, const double *y1, const double *y2, double *yn,
                             double *Tb, double *chib, int tform, int first, double mu,
                             double nu, double mut, double gamt, double dt) {
  const DiffBufs &d = c.diff;
  if (tform)
    hipLaunchKernelGGL(diff_stage_kernel<true>, dim3(grid_blocks(c)), dim3(256), 0, c.stream,
                       c.ph, c.dparams, U, Ta, chia, y0, y1, y2, d.M0, d.cv0, first, mu, nu,
                       mut, gamt, dt, yn, Tb, chib, c.flags);
  else
    hipLaunchKernelGGL(diff_stage_kernel<false>, dim3(grid_blocks(c)), dim3(256), 0, c.stream,
                       c.ph, c.dparams, U, Ta, chia, y0, y1, y2, d.M0, d.cv0, first, mu, nu,
                       mut, gamt, dt, yn, Tb, chib, c.flags);
  return hipGetLastError();
}

hipError_t launch_diff_finish(const Ctx &c, double *U, const double *ylast, const double *Tlast,
                              int tform, double *Tstore) {
  const DiffBufs &d = c.diff;
  hipLaunchKernelGGL(diff_finish_kernel, dim3(grid_blocks(c)), dim3(256), 0, c.stream, c.ph, U,
                     d.e0, ylast, Tlast, tform, Tstore);
  return hipGetLastError();
}

hipError_t launch_parabolic_dt(const Ctx &c, const double *U, const double *Bx,
                               const double *By, const double *Bz, const double *Tg,
                               double *dtp_dev) {
  int nb = (int)((c.ncell + 255) / 256);
  nb = nb < 2048 ? nb : 2048;
  hipLaunchKernelGGL(parabolic_kernel, dim3(nb), dim3(256), 0, c.stream, c.ph, c.dparams, U, Bx,
                     By, Bz, Tg, c.red, c.flags);
  hipLaunchKernelGGL(parabolic_finish_kernel, dim3(1), dim3(256), 0, c.stream, c.red, nb,
                     dtp_dev);
  return hipGetLastError();
}

}  // namespace mhd
