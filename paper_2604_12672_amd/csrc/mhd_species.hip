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
// a X^n + b X^(s) - c dt div.  One cell per thread over XCD-contiguous
// chunks; each face is evaluated by both of its cells, the stencils come
// from the caches.
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

__global__ __launch_bounds__(256) void species_kernel(Phys ph, SpeciesPtrs p, int ns, double ca,
                                                      double cb, double cc, double dt_host) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const double dt = p.dt_dev ? *p.dt_dev : dt_host;
  const double cdt = cc * dt;
  const bool pph = ph.recon == MHD_RECON_PPH;
  const double idxs[3] = {ph.idx, ph.idy, ph.idz};
  const int lens[3] = {ph.nx, ph.ny, ph.nz};
  size_t c0, c1;
  block_cells(n, c0, c1);
  for (size_t q = c0 + threadIdx.x; q < c1; q += blockDim.x) {
    int ijk[3];
    cell_ijk(ph, q, ijk[0], ijk[1], ijk[2]);
    double r[MHD_MAX_SPECIES];
#pragma unroll
    for (int l = 0; l < MHD_MAX_SPECIES; ++l) r[l] = 0.0;
    for (int axis = 0; axis < 3; ++axis) {
      // an axis of one cell carries the same face below and above the cell
      // with the same upwind values: no divergence
      if (!ph.dims_active[axis]) continue;
      const int len = lens[axis];
      const bool wall = axis == 2 && ph.reflect;
      const size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)ph.nx : plane);
      const int a0 = ijk[axis];
      const size_t base = q - (size_t)a0 * stride;  // the cell at index 0 on this line
      double fl[2];                   // mass flux / sum of fractions, per face
      double ff[2][MHD_MAX_SPECIES];  // upwind face fractions, per face
      for (int side = 0; side < 2; ++side) {
        // the face: lower (side 0) at a0 - 1/2, upper (side 1) at a0 + 1/2
        double F;
        if (axis == 0)
          F = p.mfx[base + (size_t)wrapi(a0 + side, len)];
        else if (axis == 1)
          F = p.mfy[base + (size_t)wrapi(a0 + side, len) * stride];
        else
          F = p.mfz[base + (size_t)(wall ? a0 + side : wrapi(a0 + side, len)) * stride];
        // upwind cell and which of its faces this is
        const int u = F >= 0.0 ? a0 + side - 1 : a0 + side;
        const bool upper = F >= 0.0;
        const size_t qm = base + (size_t)axis_cell(u - 1, len, wall) * stride;
        const size_t qu = base + (size_t)axis_cell(u, len, wall) * stride;
        const size_t qp = base + (size_t)axis_cell(u + 1, len, wall) * stride;
        const bool par = pph && !(p.flat && p.flat[qu]);
        const double im = rcp<double>(p.rho[qm]), iu = rcp<double>(p.rho[qu]),
                     ip = rcp<double>(p.rho[qp]);
        double sum = 0.0;
#pragma unroll
        for (int l = 0; l < MHD_MAX_SPECIES; ++l) {
          if (l < ns) {
            const double* X = p.Xs + (size_t)l * n;
            const double v = fraction_face(X[qm] * im, X[qu] * iu, X[qp] * ip, upper, par);
            ff[side][l] = v;
            sum += v;
          }
        }
        fl[side] = F * rcp<double>(sum);
      }
      const double id = idxs[axis];
#pragma unroll
      for (int l = 0; l < MHD_MAX_SPECIES; ++l)
        if (l < ns) r[l] += (fl[1] * ff[1][l] - fl[0] * ff[0][l]) * id;
    }
#pragma unroll
    for (int l = 0; l < MHD_MAX_SPECIES; ++l) {
      if (l < ns) {
        const size_t o = (size_t)l * n + q;
        double v = cb * p.Xs[o] - cdt * r[l];
        if (ca != 0.0) v += ca * p.X0[o];
        p.Xo[o] = v;
      }
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
  long long nb = (long long)((c.ncell + 255) / 256);
  nb = nb < 65536 ? nb : 65536;
  hipLaunchKernelGGL(species_kernel, dim3((unsigned)nb), dim3(256), 0, c.stream, c.ph, p,
                     c.d.nspecies, a, b, cc, dt_host);
  return hipGetLastError();
}

}  // namespace mhd
