// mhd_diffusion.hip -- thermal diffusion with RKL2 super-time-stepping
// (Sect. 2.10) on gfx950.
//
// The operator M[T] = (1/rho) div(K grad T) uses the harmonic mean of
// chi = T^3 / (kappa rho) for the face conductivity K = (4 a c / 3) chi_f
// and a power-law opacity kappa = kappa0 rho^alpha T^beta.  One kernel per
// RKL2 stage: every cell forms M from T and chi of itself and its six
// neighbours of the previous stage (two ping-pong buffers), combines the
// stage (mu, nu, mu~, gamma~ of Meyer, Balsara & Aslam), and writes its new
// value together with its new T (Newton from the previous stage's T in the
// internal-energy form; the value itself in the temperature form) and chi,
// so the next stage reads them without recomputing powers.  The stage
// kernel marches z through column tiles with the z neighbours in registers
// and the x/y neighbours in LDS; the other kernels are coalesced per-cell
// streams.
#include <hip/hip_runtime.h>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {

__device__ __forceinline__ double chi_of(const DiffParams &dp, double rho, double T) {
  // T^3 / (kappa0 rho^alpha T^beta rho) = T^(3 - beta) rho^(-1 - alpha) / kappa0
  return exp((3.0 - dp.beta) * log(T) - (1.0 + dp.alpha) * log(rho)) * dp.ikappa0;
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
//
// A block owns a 64 x 4 column tile and a z segment and marches up it: the
// column's T and chi of planes k-1, k, k+1 stay in registers (the z
// neighbours), the tile's plane k with a one-cell ring is staged in LDS
// (the x and y neighbours), so T and chi are read from HBM about once.
constexpr int DTX = 64, DTY = 4;                // tile (256 threads)
constexpr int DLX = DTX + 2, DLY = DTY + 2;     // staged plane with its ring
constexpr int DZSEG = 16;                       // planes per block

template <bool TF>
__global__ __launch_bounds__(256) void diff_stage_kernel(
    Phys ph, DiffParams dp, const double *__restrict__ U, const double *__restrict__ Ta,
    const double *__restrict__ chia, const double *__restrict__ y0,
    const double *__restrict__ y1, const double *__restrict__ y2, double *__restrict__ M0,
    const double *__restrict__ cv0, int first, double mu, double nu, double mut,
    double gamt, double dt, double *__restrict__ yn, double *__restrict__ Tb,
    double *__restrict__ chib, int *flags) {
  __shared__ double sT[DLY][DLX], sC[DLY][DLX];
  const size_t plane = (size_t)ph.nx * ph.ny;
  const double *rho = U;
  const double *yp = TF ? Ta : y1;
  const int tid = threadIdx.x;
  const int tx = tid % DTX, ty = tid / DTX;
  const int ntx = (ph.nx + DTX - 1) / DTX, nty = (ph.ny + DTY - 1) / DTY;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int btx = lb % ntx, bty = (lb / ntx) % nty, bz = lb / (ntx * nty);
  const int X0 = btx * DTX, Y0 = bty * DTY;
  const int z0 = bz * DZSEG, z1 = min(z0 + DZSEG, ph.nz);
  const int gx = X0 + tx, gy = Y0 + ty;
  const bool own = gx < ph.nx && gy < ph.ny;
  const size_t col = (size_t)wrapi(gy, ph.ny) * ph.nx + wrapi(gx, ph.nx);
  // z neighbours of the column (a wall plane's missing neighbour is never
  // used: the wall is insulating)
  auto zp = [&](int m) { return (size_t)wrapi(m, ph.nz) * plane + col; };
  double tm = Ta[zp(z0 - 1)], cm = chia[zp(z0 - 1)];
  double tc = Ta[zp(z0)], ccur = chia[zp(z0)];
  for (int k = z0; k < z1; ++k) {
    // the next plane's values are requested before this plane is evaluated
    const double tn = Ta[zp(k + 1)], cn = chia[zp(k + 1)];
    const size_t pk = (size_t)k * plane;
    sT[ty + 1][tx + 1] = tc;
    sC[ty + 1][tx + 1] = ccur;
    for (int h = tid; h < DLX * DLY - DTX * DTY; h += 256) {
      // ring cells: bottom row, top row, then left and right columns
      int hx, hy;
      if (h < DLX) {
        hy = 0;
        hx = h;
      } else if (h < 2 * DLX) {
        hy = DLY - 1;
        hx = h - DLX;
      } else {
        const int t = h - 2 * DLX;  // 0 .. 2 DTY - 1
        hy = 1 + t / 2;
        hx = (t & 1) ? DLX - 1 : 0;
      }
      const size_t qh = pk + (size_t)wrapi(Y0 - 1 + hy, ph.ny) * ph.nx + wrapi(X0 - 1 + hx, ph.nx);
      sT[hy][hx] = Ta[qh];
      sC[hy][hx] = chia[qh];
    }
    __syncthreads();
    const size_t q = pk + col;
    // M[T]: the face fluxes in the order x-, x+, y-, y+, z-, z+
    double div = 0.0;
    auto face = [&](double tnb, double cnb, double inv_dx) {
      const double K = dp.pref * 2.0 * ccur * cnb * rcp<double>(ccur + cnb);
      return K * (tnb - tc) * inv_dx * inv_dx;
    };
    if (ph.dims_active[0])
      div += face(sT[ty + 1][tx], sC[ty + 1][tx], ph.idx) +
             face(sT[ty + 1][tx + 2], sC[ty + 1][tx + 2], ph.idx);
    if (ph.dims_active[1])
      div += face(sT[ty][tx + 1], sC[ty][tx + 1], ph.idy) +
             face(sT[ty + 2][tx + 1], sC[ty + 2][tx + 1], ph.idy);
    if (ph.dims_active[2]) {
      if (!(ph.reflect && k == 0)) div += face(tm, cm, ph.idz);
      if (!(ph.reflect && k + 1 == ph.nz)) div += face(tn, cn, ph.idz);
    }
    if (own) {
      const double r = rho[q];
      double M = div * rcp<double>(r);
      if (TF) M *= rcp<double>(cv0[q]);
      double v;
      if (first) {
        M0[q] = M;
        v = y0[q] + mut * dt * M;
      } else {
        v = mu * yp[q] + nu * y2[q] + (1.0 - mu - nu) * y0[q] + mut * dt * M +
            gamt * dt * M0[q];
      }
      yn[q] = v;
      double t = v;
      if (!TF) {
        int it, fb;
        if (!(v > 0.0) || eos_temperature(ph, r, v, tc, ph.newton_maxit, t, it, fb))
          atomicOr(flags, 2);
        Tb[q] = t;
      } else if (!(v > 0.0)) {
        atomicOr(flags, 2);
      }
      chib[q] = chi_of(dp, r, t);
    }
    __syncthreads();
    tm = tc;
    cm = ccur;
    tc = tn;
    ccur = cn;
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
  const dim3 grid(((c.ph.nx + DTX - 1) / DTX) * ((c.ph.ny + DTY - 1) / DTY) *
                  ((c.ph.nz + DZSEG - 1) / DZSEG));
  if (tform)
    hipLaunchKernelGGL(diff_stage_kernel<true>, grid, dim3(256), 0, c.stream,
                       c.ph, c.dparams, U, Ta, chia, y0, y1, y2, d.M0, d.cv0, first, mu, nu,
                       mut, gamt, dt, yn, Tb, chib, c.flags);
  else
    hipLaunchKernelGGL(diff_stage_kernel<false>, grid, dim3(256), 0, c.stream,
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
