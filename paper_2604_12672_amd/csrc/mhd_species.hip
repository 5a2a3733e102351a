// mhd_species.hip -- passive species (Sect. 2.9, consistent multi-fluid
// advection) on gfx950.
//
// The stage kernel writes the mass flux of every face it owns (the lower x,
// y and z faces of its cells, plus the top wall).  This kernel then advances
// the partial densities rho X_l of the same RK stage: per cell and face it
// takes the upwind side of the mass flux (the cell below the face when the
// flux is >= 0, else the cell above; for HLLC/HLLD this is the side of the
// contact that holds the face), reconstructs that cell's mass fractions at
// the face (van Leer, or in PPH mode the three-cell parabola bounded by the
// averages beside each face and made monotone after Colella & Woodward;
// van Leer in flattened cells), rescales them to sum to one, and
// accumulates flux x fraction.  The update is the stage's combination
// a X^n + b X^(s) - c dt div.  One cell per thread; each face is evaluated
// by both of its cells, the stencils come from the caches.
#include <hip/hip_runtime.h>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {

struct SpeciesPtrs {
  const double *rho;               // stage input density U^(s)[0]
  const double *Xs;                // stage input rho X_l [ns][n]
  const double *X0;                // step base rho X_l (read when a != 0)
  double *Xo;                      // stage output
  const double *mfx, *mfy, *mfz;   // face mass fluxes of this stage
  const uint8_t *flat;             // flattening flags (nullable)
  const double *dt_dev;            // device dt (nullable)
};

__device__ __forceinline__ double clamp_between(double v, double a, double b) {
  const double lo = fmin(a, b), hi = fmax(a, b);
  return fmin(fmax(v, lo), hi);
}

// Face value of one mass fraction from the cell and its two neighbours along
// the axis: upper face (hi) or lower face.  Van Leer, or the limited parabola.
__device__ __forceinline__ double fraction_face(double xm, double xc, double xp, bool upper,
                                                bool parabola) {
  if (!parabola) {
    const double s = 0.5 * vanleer<double>(xc - xm, xp - xc);
    return upper ? xc + s : xc - s;
  }
  double l = (2.0 * xm + 5.0 * xc - xp) * (1.0 / 6.0);
  double h = (5.0 * xc - xm + 2.0 * xp) * (1.0 / 6.0);
  l = clamp_between(l, xm, xc);
  h = clamp_between(h, xc, xp);
  if ((h - xc) * (xc - l) <= 0.0) {
    l = xc;
    h = xc;
  } else {
    const double d = h - l;
    const double m6 = 6.0 * (xc - 0.5 * (l + h));
    if (d * m6 > d * d)
      l = 3.0 * xc - 2.0 * h;
    else if (-d * d > d * m6)
      h = 3.0 * xc - 2.0 * l;
  }
  return upper ? h : l;
}

// index of cell a along an axis of n cells: periodic, or the mirror image
// across a wall (mass fractions and density are even)
__device__ __forceinline__ int axis_cell(int a, int n, bool wall) {
  if (!wall) return wrapi(a, n);
  if (a < 0) return -1 - a;
  if (a >= n) return 2 * n - 1 - a;
  return a;
}

// One block per 16 x 16 tile of one plane.  Each face's
// fractions are used as soon as they are reconstructed, so the registers
// hold the accumulators and one face's fractions (NS each).
constexpr int SP_T = 16;  // tile edge (256 threads)

template <int NS>
__global__ __launch_bounds__(256) void species_kernel(Phys ph, SpeciesPtrs p, int ns, double ca,
                                                      double cb, double cc, double dt_host) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const double dt = p.dt_dev ? *p.dt_dev : dt_host;
  const double cdt = cc * dt;
  const bool pph = ph.recon == MHD_RECON_PPH;
  // logical order: x tiles fastest, then planes, then rows of tiles, so the
  // blocks in flight on one XCD cover whole rows of tiles over a few planes
  // (x halos and z stencils come from L2)
  const int ntx = (ph.nx + SP_T - 1) / SP_T;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int btx = lb % ntx, rest = lb / ntx;
  const int kk = rest % ph.nz, bty = rest / ph.nz;
  const int ii = btx * SP_T + (int)(threadIdx.x % SP_T);
  const int jj = bty * SP_T + (int)(threadIdx.x / SP_T);
  if (ii >= ph.nx || jj >= ph.ny) return;
  const size_t q = (size_t)kk * plane + (size_t)jj * ph.nx + ii;
  const int ijk[3] = {ii, jj, kk};
  const int lens[3] = {ph.nx, ph.ny, ph.nz};
  const double idxs[3] = {ph.idx, ph.idy, ph.idz};
  double r[NS];
#pragma unroll
  for (int l = 0; l < NS; ++l) r[l] = 0.0;
  // every loop below is unrolled, so the per-species arrays stay in
  // registers (an index the compiler cannot resolve would put them in
  // scratch memory)
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    // an axis of one cell carries the same face below and above the cell
    // with the same upwind values: no divergence
    if (!ph.dims_active[axis]) continue;
    const int len = lens[axis];
    const bool wall = axis == 2 && ph.reflect;
    const size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)ph.nx : plane);
    const int a0 = ijk[axis];
    const size_t base = q - (size_t)a0 * stride;  // the cell at index 0 on this line
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      // the face: lower (side 0) at a0 - 1/2, upper (side 1) at a0 + 1/2
      const double *mf = axis == 0 ? p.mfx : (axis == 1 ? p.mfy : p.mfz);
      const int fa = wall ? a0 + side : wrapi(a0 + side, len);
      const double F = mf[base + (size_t)fa * stride];
      // upwind cell and which of its faces this is
      const int u = F >= 0.0 ? a0 + side - 1 : a0 + side;
      const bool upper = F >= 0.0;
      const size_t qm = base + (size_t)axis_cell(u - 1, len, wall) * stride;
      const size_t qu = base + (size_t)axis_cell(u, len, wall) * stride;
      const size_t qp = base + (size_t)axis_cell(u + 1, len, wall) * stride;
      const bool par = pph && !(p.flat && p.flat[qu]);
      const double im = rcp<double>(p.rho[qm]), iu = rcp<double>(p.rho[qu]),
                   ip = rcp<double>(p.rho[qp]);
      double v[NS];
      double sum = 0.0;
#pragma unroll
      for (int l = 0; l < NS; ++l) {
        v[l] = 0.0;
        if (l < ns) {
          const double *X = p.Xs + (size_t)l * n;
          v[l] = fraction_face(X[qm] * im, X[qu] * iu, X[qp] * ip, upper, par);
          sum += v[l];
        }
      }
      // flux of species l: F v_l / sum, entering the divergence with the
      // face's sign
      const double g = (side ? F : -F) * rcp<double>(sum) * idxs[axis];
#pragma unroll
      for (int l = 0; l < NS; ++l)
        if (l < ns) r[l] += g * v[l];
    }
  }
#pragma unroll
  for (int l = 0; l < NS; ++l) {
    if (l < ns) {
      const size_t o = (size_t)l * n + q;
      double val = cb * p.Xs[o] - cdt * r[l];
      if (ca != 0.0) val += ca * p.X0[o];
      p.Xo[o] = val;
    }
  }
}

hipError_t launch_species(const Ctx &c, const double *rho, const double *Xs, const double *X0,
                          double *Xo, double a, double b, double cc, double dt_host,
                          const double *dt_dev, const uint8_t *flat) {
  SpeciesPtrs p;
  p.rho = rho;
  p.Xs = Xs;
  p.X0 = X0;
  p.Xo = Xo;
  p.mfx = c.mf[0];
  p.mfy = c.mf[1];
  p.mfz = c.mf[2];
  p.flat = flat;
  p.dt_dev = dt_dev;
  const int ns = c.d.nspecies;
  const dim3 grid(((c.ph.nx + SP_T - 1) / SP_T) * ((c.ph.ny + SP_T - 1) / SP_T) * c.ph.nz);
  // register arrays sized for the species count (a few variants)
  if (ns <= 4)
    hipLaunchKernelGGL(species_kernel<4>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host);
  else if (ns <= 8)
    hipLaunchKernelGGL(species_kernel<8>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host);
  else if (ns <= 12)
    hipLaunchKernelGGL(species_kernel<12>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host);
  else
    hipLaunchKernelGGL(species_kernel<16>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host);
  return hipGetLastError();
}

}  // namespace mhd
