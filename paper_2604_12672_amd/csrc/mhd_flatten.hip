// mhd_flatten.hip -- shock-flattening flags (Sect. 2.7) on gfx950.
//
// Before each RK stage with flattening enabled:
//   shock_pressure_kernel  thermal pressure P of every cell of the stage
//                          input (the EOS inversion from the stage's guess,
//                          as the stage itself does it);
//   shock_detect_kernel    detector (|P_{i+1} - P_{i-1}| + |P_{j+1} - P_{j-1}|
//                          + |P_{k+1} - P_{k-1}|) / (eps_SF P) > 1, one byte
//                          per cell; neighbours periodic in x, y (and z), the
//                          mirror image (the cell itself) at a wall;
//   shock_dilate_kernel    OR over two cells either side along one axis, run
//                          for x, y and z: the 5x5x5 dilation, cut off at a
//                          wall (a mirror image only repeats cells inside).
// The stage kernel reads the final byte per cell.  Every kernel is a
// coalesced per-cell stream with the stencil neighbours from the caches.
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

__global__ __launch_bounds__(256) void shock_detect_kernel(Phys ph, double eps,
                                                           const double *__restrict__ P,
                                                           uint8_t *__restrict__ det) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  size_t c0, c1;
  block_cells(n, c0, c1);
  for (size_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const size_t row = q - i, pl = q - (size_t)k * plane;
    const int im = i == 0 ? ph.nx - 1 : i - 1, ip = i + 1 == ph.nx ? 0 : i + 1;
    const int jm = j == 0 ? ph.ny - 1 : j - 1, jp = j + 1 == ph.ny ? 0 : j + 1;
    int km, kp;
    if (ph.reflect) {
      km = k == 0 ? 0 : k - 1;
      kp = k + 1 == ph.nz ? k : k + 1;
    } else {
      km = k == 0 ? ph.nz - 1 : k - 1;
      kp = k + 1 == ph.nz ? 0 : k + 1;
    }
    const size_t colj = q - (size_t)j * ph.nx;  // cell (i, 0, k)
    const double sum = fabs(P[row + ip] - P[row + im]) +
                       fabs(P[colj + (size_t)jp * ph.nx] - P[colj + (size_t)jm * ph.nx]) +
                       fabs(P[(size_t)kp * plane + pl] - P[(size_t)km * plane + pl]);
    // the decision in IEEE double, as written: sum / (eps P) > 1
    det[q] = sum / (eps * P[q]) > 1.0 ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void shock_dilate_kernel(Phys ph, int axis,
                                                           const uint8_t *__restrict__ in,
                                                           uint8_t *__restrict__ out) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const int len = axis == 0 ? ph.nx : (axis == 1 ? ph.ny : ph.nz);
  const size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)ph.nx : plane);
  const bool cut = axis == 2 && ph.reflect;
  size_t c0, c1;
  block_cells(n, c0, c1);
  for (size_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const int a = axis == 0 ? i : (axis == 1 ? j : k);
    const size_t base = q - (size_t)a * stride;
    uint8_t f = 0;
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
      int b = a + d;
      if (cut) {
        if (b < 0 || b >= len) continue;
      } else {
        b = wrapi(b, len);
      }
      f |= in[base + (size_t)b * stride];
    }
    out[q] = f;
  }
}

static int flat_blocks(const Ctx &c) {
  long long nb = (long long)((c.ncell + 255) / 256);
  return (int)(nb < 65536 ? nb : 65536);
}

hipError_t launch_shock_flags(const Ctx &c, const double *U, const double *Bx, const double *By,
                              const double *Bz, const double *Tg, int newton_cap) {
  const dim3 grid(flat_blocks(c)), block(256);
  if (c.ph.gasrad)
    hipLaunchKernelGGL(shock_pressure_kernel<true>, grid, block, 0, c.stream, c.ph, U, Bx, By, Bz,
                       Tg, newton_cap, c.shock_p, c.flags);
  else
    hipLaunchKernelGGL(shock_pressure_kernel<false>, grid, block, 0, c.stream, c.ph, U, Bx, By,
                       Bz, nullptr, newton_cap, c.shock_p, c.flags);
  hipLaunchKernelGGL(shock_detect_kernel, grid, block, 0, c.stream, c.ph, c.d.eps_sf, c.shock_p,
                     c.shock_f[0]);
  // x: f0 -> f1, y: f1 -> f0, z: f0 -> f1
  hipLaunchKernelGGL(shock_dilate_kernel, grid, block, 0, c.stream, c.ph, 0, c.shock_f[0],
                     c.shock_f[1]);
  hipLaunchKernelGGL(shock_dilate_kernel, grid, block, 0, c.stream, c.ph, 1, c.shock_f[1],
                     c.shock_f[0]);
  hipLaunchKernelGGL(shock_dilate_kernel, grid, block, 0, c.stream, c.ph, 2, c.shock_f[0],
                     c.shock_f[1]);
  return hipGetLastError();
}

}  // namespace mhd
