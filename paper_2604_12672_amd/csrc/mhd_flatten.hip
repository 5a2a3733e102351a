// mhd_flatten.hip -- shock-flattening flags (Sect. 2.7) on gfx950.
//
// Before each RK stage with flattening enabled:
//   shock_pressure_kernel  thermal pressure P of every cell of the stage
//                          input (the EOS inversion from the stage's guess,
//                          as the stage itself does it);
//   shock_flag_kernel      detector (|P_{i+1} - P_{i-1}| + |P_{j+1} - P_{j-1}|
//                          + |P_{k+1} - P_{k-1}|) / (eps_SF P) > 1 with the
//                          neighbours periodic in x, y (and z) and the mirror
//                          image (the cell itself) at a wall, and its OR over
//                          two cells either side along every axis (the 5x5x5
//                          dilation, cut off at a wall, where a mirror image
//                          only repeats cells inside), one byte per cell.
// The stage kernel reads the byte of every cell it reconstructs.
#include <hip/hip_runtime.h>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {

template <bool GR>
__global__ __launch_bounds__(256) void shock_pressure_kernel(
    Phys ph, const double *__restrict__ U, const double *__restrict__ Bx,
    const double *__restrict__ By, const double *__restrict__ Bz,
    const double *__restrict__ Tg, int maxit, double *__restrict__ P, int *flags) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const double zero_bg[4] = {0.0, 0.0, 0.0, 0.0};
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
    PrimOut o;
    cons2prim<GR>(ph, u, b, Tg ? Tg[q] : 0.0, zero_bg, o, maxit);
    if (o.bad) atomicOr(flags, o.bad);
    P[q] = o.w[Q_P];  // full pressure: the background passed is zero
  }
}

// Detector and dilation in one pass.  A block owns a 16 x 16 column tile and
// a z segment and marches up it.  Per plane it stages the pressure of the
// tile with a three-cell halo in LDS (a ring of three planes), evaluates the
// detector on the tile with a two-cell halo, ORs it over five cells along x
// and then along y, and keeps the last five planes of that in registers:
// the OR over them is the dilated flag of the plane two below.  The square
// tile evaluates the detector on 1.56 times its cells and loads 1.9 times
// its pressures per plane (2.1 and 2.7 times for a 64 x 4 tile).
constexpr int FX = 16, FY = 16;           // output tile (256 threads)
constexpr int PX = FX + 6, PY = FY + 6;   // pressure tile (halo 3)
constexpr int DX = FX + 4, DY = FY + 4;   // detector tile (halo 2)
constexpr int FZSEG = 32;                 // planes per block

__global__ __launch_bounds__(256) void shock_flag_kernel(Phys ph, double eps,
                                                         const double *__restrict__ P,
                                                         uint8_t *__restrict__ out) {
  __shared__ double sP[3][PY][PX];
  __shared__ uint8_t sD[DY][DX];
  __shared__ uint8_t sX[DY][FX];
  const int tid = threadIdx.x;
  const int tx = tid % FX, ty = tid / FX;
  const int ntx = (ph.nx + FX - 1) / FX, nty = (ph.ny + FY - 1) / FY;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int btx = lb % ntx, bty = (lb / ntx) % nty, bz = lb / (ntx * nty);
  const int X0 = btx * FX, Y0 = bty * FY;
  const int z0 = bz * FZSEG, z1 = min(z0 + FZSEG, ph.nz);
  const size_t plane = (size_t)ph.nx * ph.ny;
  const int gx = X0 + tx, gy = Y0 + ty;
  const bool own = gx < ph.nx && gy < ph.ny;

  // pressure plane kp, fetched into registers one plane ahead (three
  // values per thread) and stored into its LDS ring slot at the top of the
  // next plane; below / above a wall the mirror image (P is even), else the
  // periodic image.  The clamp only touches planes three beyond a wall,
  // which feed no detector plane that is used.
  constexpr int PER = (PX * PY + 255) / 256;
  double pre[PER];
  auto fetch_plane = [&](int kp) {
    int kk;
    if (ph.reflect) {
      kk = kp < 0 ? -1 - kp : (kp >= ph.nz ? 2 * ph.nz - 1 - kp : kp);
      kk = kk < 0 ? 0 : (kk >= ph.nz ? ph.nz - 1 : kk);
    } else {
      kk = wrapi(kp, ph.nz);
    }
    const double *src = P + (size_t)kk * plane;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + m * 256;
      if (idx < PX * PY) {
        const int r = idx / PX, c = idx - r * PX;
        const int xx = wrapi(X0 - 3 + c, ph.nx), yy = wrapi(Y0 - 3 + r, ph.ny);
        pre[m] = src[(size_t)yy * ph.nx + xx];
      }
    }
  };
  auto store_plane = [&](int kp) {
    double(*dst)[PX] = sP[wrapi(kp, 3)];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int idx = tid + m * 256;
      if (idx < PX * PY) {
        const int r = idx / PX, c = idx - r * PX;
        dst[r][c] = pre[m];
      }
    }
  };
  fetch_plane(z0 - 3);
  store_plane(z0 - 3);
  fetch_plane(z0 - 2);
  store_plane(z0 - 2);
  fetch_plane(z0 - 1);
  uint8_t ring[5] = {0, 0, 0, 0, 0};  // x/y-dilated detector, planes kd-4 .. kd
  for (int kd = z0 - 2; kd <= z1 + 1; ++kd) {
    store_plane(kd + 1);
    __syncthreads();
    if (kd <= z1) fetch_plane(kd + 2);  // in flight while this plane is evaluated
    // detector planes beyond a wall do not exist (the dilation is cut there)
    const bool valid = !(ph.reflect && (kd < 0 || kd >= ph.nz));
    if (valid) {
      const double(*pm)[PX] = sP[wrapi(kd - 1, 3)];
      const double(*pc)[PX] = sP[wrapi(kd, 3)];
      const double(*pp)[PX] = sP[wrapi(kd + 1, 3)];
      for (int idx = tid; idx < DX * DY; idx += 256) {
        const int r = idx / DX, c = idx - r * DX;
        const int pr = r + 1, pcl = c + 1;  // the same cell in the pressure tile
        const double sum = fabs(pc[pr][pcl + 1] - pc[pr][pcl - 1]) +
                           fabs(pc[pr + 1][pcl] - pc[pr - 1][pcl]) +
                           fabs(pp[pr][pcl] - pm[pr][pcl]);
        // sum / (eps P) > 1 of the paper, decided without the division: for
        // finite positive doubles x, y the correctly rounded x / y exceeds 1
        // exactly when x > y (x > y means x >= y + ulp(y) > y (1 + 2^-53),
        // whose quotient rounds above 1)
        sD[r][c] = sum > eps * pc[pr][pcl] ? 1 : 0;
      }
    }
    __syncthreads();
    if (valid) {
      for (int idx = tid; idx < DY * FX; idx += 256) {
        const int r = idx / FX, c = idx - r * FX;
        sX[r][c] = sD[r][c] | sD[r][c + 1] | sD[r][c + 2] | sD[r][c + 3] | sD[r][c + 4];
      }
    }
    __syncthreads();
    const uint8_t xy = valid ? (uint8_t)(sX[ty][tx] | sX[ty + 1][tx] | sX[ty + 2][tx] |
                                         sX[ty + 3][tx] | sX[ty + 4][tx])
                             : (uint8_t)0;
#pragma unroll
    for (int i = 0; i < 4; ++i) ring[i] = ring[i + 1];
    ring[4] = xy;
    if (kd >= z0 + 2 && own)
      out[(size_t)(kd - 2) * plane + (size_t)gy * ph.nx + gx] =
          ring[0] | ring[1] | ring[2] | ring[3] | ring[4];
  }
}

static int flat_blocks(const Ctx &c) {
  long long nb = (long long)((c.ncell + 255) / 256);
  return (int)(nb < 65536 ? nb : 65536);
}

hipError_t launch_shock_pressure(const Ctx &c, const double *U, const double *Bx,
                                 const double *By, const double *Bz, const double *Tg,
                                 int newton_cap) {
  const dim3 grid(flat_blocks(c)), block(256);
  if (c.ph.gasrad)
    hipLaunchKernelGGL(shock_pressure_kernel<true>, grid, block, 0, c.stream, c.ph, U, Bx, By, Bz,
                       Tg, newton_cap, c.shock_p, c.flags);
  else
    hipLaunchKernelGGL(shock_pressure_kernel<false>, grid, block, 0, c.stream, c.ph, U, Bx, By,
                       Bz, nullptr, newton_cap, c.shock_p, c.flags);
  return hipGetLastError();
}

hipError_t launch_shock_flags(const Ctx &c) {
  const int nb = ((c.ph.nx + FX - 1) / FX) * ((c.ph.ny + FY - 1) / FY) *
                 ((c.ph.nz + FZSEG - 1) / FZSEG);
  hipLaunchKernelGGL(shock_flag_kernel, dim3(nb), dim3(256), 0, c.stream, c.ph, c.d.eps_sf,
                     c.shock_p, c.shock_f);
  return hipGetLastError();
}

}  // namespace mhd
