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
// a X^n + b X^(s) - c dt div.  Blocks march up column tiles (see
// species_kernel below).
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
  // the three cases without branches (the lanes of a wave rarely agree)
  const bool ext = (h - xc) * (xc - l) <= 0.0;
  const double d = h - l;
  const double m6 = 6.0 * (xc - 0.5 * (l + h));
  const bool lo_over = d * m6 > d * d;
  const bool hi_over = !lo_over && -d * d > d * m6;
  const double lf = ext ? xc : (lo_over ? 3.0 * xc - 2.0 * h : l);
  const double hf = ext ? xc : (hi_over ? 3.0 * xc - 2.0 * l : h);
  return upper ? hf : lf;
}

// index of cell a along an axis of n cells: periodic, or the mirror image
// across a wall (mass fractions and density are even)
__device__ __forceinline__ int axis_cell(int a, int n, bool wall) {
  if (!wall) return wrapi(a, n);
  if (a < 0) return -1 - a;
  if (a >= n) return 2 * n - 1 - a;
  return a;
}

// Access through a block-uniform base pointer and a 32-bit per-lane byte
// offset (a plane is below 4 GiB: checked at launch).
__device__ __forceinline__ double ldu(const double *base, unsigned off) {
  return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + off);
}
__device__ __forceinline__ void stu(double *base, unsigned off, double v) {
  *reinterpret_cast<double *>(reinterpret_cast<char *>(base) + off) = v;
}

// The value held by the other lane of this lane's pair (lanes 2m, 2m+1):
// DPP quad_perm [1,0,3,2].  Must be called with all lanes active.
__device__ __forceinline__ double pair_other(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// One block per 16 x 8 column tile and z segment; it marches up the
// segment one plane at a time.  Two lanes of a pair share a column, each
// with half of the species, and add their sums of face fractions over the
// pair (a + b on one lane, b + a on the other: the same number).  Each lane
// keeps its species' partial densities and 1/rho of its column for planes
// k-1 .. k+2 in registers (the z stencils of both possible upwind cells of
// the face k+1/2); the block stages the mass fractions of plane k with a
// two-cell halo in LDS for the x and y stencils.  The z-face k+1/2 is
// evaluated once per column and enters cells k and k+1; the x and y faces
// are evaluated by both of their cells.  Every loop over species is
// unrolled, so the per-species arrays stay in registers.
constexpr int SP_TX = 16, SP_TY = 8;                          // columns per tile
constexpr int SP_HX = SP_TX + 4, SP_HY = SP_TY + 4;           // staged plane
constexpr int SP_HALO = SP_HX * SP_HY - SP_TX * SP_TY;        // 112 halo cells
constexpr int SP_ZSEG = 32;                                   // planes per block

// LDS position of halo cell h (0 <= h < SP_HALO): the two rows below and
// above the tile (full width), then the two columns either side
__device__ __forceinline__ int halo_pos(int h) {
  if (h < 2 * SP_HX) return h;
  h -= 2 * SP_HX;
  if (h < 2 * SP_HX) return (SP_HY - 2) * SP_HX + h;
  h -= 2 * SP_HX;
  const int c = h & 3;
  return (2 + (h >> 2)) * SP_HX + (c < 2 ? c : SP_HX - 4 + c);
}

template <int NH>  // species per lane (the pair holds 2 NH)
__global__ __launch_bounds__(256) void species_kernel(Phys ph, SpeciesPtrs p, int ns, double ca,
                                                      double cb, double cc, double dt_host,
                                                      int zseg) {
  __shared__ double sX[2 * NH][SP_HX * SP_HY];  // mass fractions of plane k
  __shared__ unsigned char sFl[SP_HX * SP_HY];  // flattening flags of plane k
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const double dt = p.dt_dev ? *p.dt_dev : dt_host;
  const double cdt = cc * dt;
  const bool pph = ph.recon == MHD_RECON_PPH;
  const bool wall = ph.reflect != 0;
  const bool base = ca != 0.0;
  // an axis of one cell carries the same face below and above the cell
  // with the same upwind values: no divergence
  const bool xa = ph.dims_active[0], ya = ph.dims_active[1], za = ph.dims_active[2];
  // logical order: x tiles fastest, then y tiles, then z segments (each XCD
  // walks a contiguous run: neighbouring tiles march up the same planes)
  const int ntx = (ph.nx + SP_TX - 1) / SP_TX, nty = (ph.ny + SP_TY - 1) / SP_TY;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int btx = lb % ntx, bty = (lb / ntx) % nty, bsz = lb / (ntx * nty);
  const int X0 = btx * SP_TX, Y0 = bty * SP_TY;
  const int z0 = bsz * zseg, z1 = min(z0 + zseg, ph.nz);
  const int half = (int)(threadIdx.x & 1), col = (int)(threadIdx.x >> 1);
  const int l0 = half * NH;  // first species of this lane
  const int tx = col % SP_TX, ty = col / SP_TX;
  const int gx = X0 + tx, gy = Y0 + ty;
  const bool own = gx < ph.nx && gy < ph.ny;
  // lanes past a ragged edge stage the periodic image of their column
  const int gi = wrapi(gx, ph.nx), gj = wrapi(gy, ph.ny);
  const unsigned colq = (unsigned)(gj * ph.nx + gi);
  const unsigned offq = colq * 8u;
  const unsigned offx = (unsigned)(gj * ph.nx + wrapi(gx + 1, ph.nx)) * 8u;  // upper x face
  const unsigned offy = (unsigned)(wrapi(gy + 1, ph.ny) * ph.nx + gi) * 8u;  // upper y face
  const int lpos = (ty + 2) * SP_HX + (tx + 2);
  // halo cell staged by this lane pair (pairs 0 .. SP_HALO-1)
  const bool hal = col < SP_HALO;
  const int hpos = hal ? halo_pos(col) : 0;
  const unsigned hcol = (unsigned)(wrapi(Y0 - 2 + hpos / SP_HX, ph.ny) * ph.nx +
                                   wrapi(X0 - 2 + hpos % SP_HX, ph.nx));

  // own column, planes k-1 .. k+2: rho X_l of this lane's species, 1/rho,
  // flag (slots 0..3)
  double w[4][NH], wir[4];
  int wf[4];
  auto zplane = [&](int a) -> size_t {
    return (size_t)(za ? axis_cell(a, ph.nz, wall) : 0) * plane;
  };
  auto load_col = [&](double *ws, double &ir, int &fl, int a) {
    const size_t zp = zplane(a);
    ir = rcp<double>(ldu(p.rho + zp, offq));
#pragma unroll
    for (int j = 0; j < NH; ++j)
      ws[j] = l0 + j < ns ? ldu(p.Xs + (size_t)(l0 + j) * n + zp, offq) : 0.0;
    fl = p.flat ? p.flat[zp + colq] : 0;
  };
  auto shift = [&]() {
#pragma unroll
    for (int s = 0; s < 3; ++s) {
#pragma unroll
      for (int j = 0; j < NH; ++j) w[s][j] = w[s + 1][j];
      wir[s] = wir[s + 1];
      wf[s] = wf[s + 1];
    }
  };
  // z-face between planes k and k+1 (slots 0..3 hold k-1 .. k+2): the
  // divergence term of cell k's upper face in t (cell k+1 takes -t)
  auto zflux = [&](int k) -> double {
    const int fa = wall ? k + 1 : wrapi(k + 1, ph.nz);
    return ldu(p.mfz + (size_t)fa * plane, offq);
  };
  auto zface = [&](double F, double *t) {
    const bool up = F >= 0.0;  // upwind: cell k (its upper face), else k+1
    const bool par = pph && !(up ? wf[1] : wf[2]);
    const double im = up ? wir[0] : wir[1], ic = up ? wir[1] : wir[2],
                 ip = up ? wir[2] : wir[3];
    double sum = 0.0;
    // one branch per face on the reconstruction (the same for all species)
    auto faces = [&](bool parabola) {
#pragma unroll
      for (int j = 0; j < NH; ++j) {
        // a species past ns is zero in every slot, so its face value is zero
        t[j] = fraction_face((up ? w[0][j] : w[1][j]) * im, (up ? w[1][j] : w[2][j]) * ic,
                             (up ? w[2][j] : w[3][j]) * ip, up, parabola);
        sum += t[j];
      }
    };
    if (par)
      faces(true);
    else
      faces(false);
    sum += pair_other(sum);
    const double g = F * rcp<double>(sum) * ph.idz;
#pragma unroll
    for (int j = 0; j < NH; ++j) t[j] = g * t[j];
  };
  double r[NH];
  // x or y face of the own cell (side 0: lower, 1: upper) from the staged
  // plane; its divergence term goes into r
  auto xyface = [&](int stride, int side, double F, double idd) {
    const bool up = F >= 0.0;
    const int c = lpos + ((up ? side - 1 : side) * stride);  // upwind cell
    const bool par = pph && !sFl[c];
    double v[NH];
    double sum = 0.0;
    // one branch per face on the reconstruction (the same for all species)
    auto faces = [&](bool parabola) {
#pragma unroll
      for (int j = 0; j < NH; ++j) {
        // rows past ns hold zeros: their face value is zero
        const double *x = sX[l0 + j];
        v[j] = fraction_face(x[c - stride], x[c], x[c + stride], up, parabola);
        sum += v[j];
      }
    };
    if (par)
      faces(true);
    else
      faces(false);
    sum += pair_other(sum);
    const double g = (side ? F : -F) * rcp<double>(sum) * idd;
#pragma unroll
    for (int j = 0; j < NH; ++j) r[j] += g * v[j];
  };

  // the halo cell of the next plane to stage, requested a plane ahead
  double hx[NH], hir = 0.0;
  int hfl = 0;
  auto load_halo = [&](int k) {
    const size_t zp = zplane(k);
    const unsigned offh = hcol * 8u;
    hir = rcp<double>(ldu(p.rho + zp, offh));
#pragma unroll
    for (int j = 0; j < NH; ++j)
      hx[j] = l0 + j < ns ? ldu(p.Xs + (size_t)(l0 + j) * n + zp, offh) : 0.0;
    hfl = p.flat ? p.flat[zp + hcol] : 0;
  };
  if (hal) load_halo(z0);
  load_col(w[0], wir[0], wf[0], z0 - 2);
  load_col(w[1], wir[1], wf[1], z0 - 1);
  load_col(w[2], wir[2], wf[2], z0);
  load_col(w[3], wir[3], wf[3], z0 + 1);
  // mass fluxes of the faces of plane k (lower and upper x and y faces,
  // upper z face), requested a plane ahead
  double fxl = 0.0, fxu = 0.0, fyl = 0.0, fyu = 0.0, fzu = 0.0;
  auto load_flux = [&](int k) {
    const size_t pk = (size_t)k * plane;
    if (xa) {
      fxl = ldu(p.mfx + pk, offq);
      fxu = ldu(p.mfx + pk, offx);
    }
    if (ya) {
      fyl = ldu(p.mfy + pk, offq);
      fyu = ldu(p.mfy + pk, offy);
    }
    if (za) fzu = zflux(k);
  };
  {
    double t[NH];
    if (za) zface(zflux(z0 - 1), t);
#pragma unroll
    for (int j = 0; j < NH; ++j) r[j] = za ? -t[j] : 0.0;
  }
  shift();
  load_flux(z0);
  for (int k = z0; k < z1; ++k) {
    // requested at the top of the plane: the column's plane k+2 (used by
    // the z-face at the end)
    load_col(w[3], wir[3], wf[3], k + 2);
    const size_t pk = (size_t)k * plane;
    const double Fxl = fxl, Fxu = fxu, Fyl = fyl, Fyu = fyu, Fzu = fzu;
    if (k + 1 < z1) load_flux(k + 1);
    // stage plane k: the own column from the registers, one halo cell
    // every row of the lane's species, the absent ones (zero) included, so
    // that the face values read from them are exactly zero
#pragma unroll
    for (int j = 0; j < NH; ++j) sX[l0 + j][lpos] = w[1][j] * wir[1];
    if (!half) sFl[lpos] = (unsigned char)wf[1];
    if (hal) {
#pragma unroll
      for (int j = 0; j < NH; ++j) sX[l0 + j][hpos] = hx[j] * hir;
      if (!half) sFl[hpos] = (unsigned char)hfl;
      if (k + 1 < z1) load_halo(k + 1);
    }
    // the base state of the update, requested before the faces
    double x0[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j)
      x0[j] = (base && own && l0 + j < ns) ? ldu(p.X0 + (size_t)(l0 + j) * n + pk, offq) : 0.0;
    __syncthreads();
    if (xa) {
      xyface(1, 0, Fxl, ph.idx);
      xyface(1, 1, Fxu, ph.idx);
    }
    if (ya) {
      xyface(SP_HX, 0, Fyl, ph.idy);
      xyface(SP_HX, 1, Fyu, ph.idy);
    }
    double t[NH];
    if (za) {
      zface(Fzu, t);
#pragma unroll
      for (int j = 0; j < NH; ++j) r[j] += t[j];
    }
    if (own) {
#pragma unroll
      for (int j = 0; j < NH; ++j) {
        if (l0 + j < ns) {
          double val = cb * w[1][j] - cdt * r[j];
          if (base) val += ca * x0[j];
          stu(p.Xo + (size_t)(l0 + j) * n + pk, offq, val);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NH; ++j) r[j] = za ? -t[j] : 0.0;
    shift();
    __syncthreads();  // plane k's stage is read before plane k+1 replaces it
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
  const int zseg = SP_ZSEG;
  // per-lane offsets within a plane are 32-bit byte offsets
  if ((unsigned long long)c.ph.nx * c.ph.ny * sizeof(double) >= (1ull << 32))
    return hipErrorInvalidValue;
  const dim3 grid(((c.ph.nx + SP_TX - 1) / SP_TX) * ((c.ph.ny + SP_TY - 1) / SP_TY) *
                  ((c.ph.nz + zseg - 1) / zseg));
  // register arrays sized for the species count (a few variants)
  if (ns <= 4)
    hipLaunchKernelGGL(species_kernel<2>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host, zseg);
  else if (ns <= 8)
    hipLaunchKernelGGL(species_kernel<4>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host, zseg);
  else if (ns <= 12)
    hipLaunchKernelGGL(species_kernel<6>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host, zseg);
  else
    hipLaunchKernelGGL(species_kernel<8>, grid, dim3(256), 0, c.stream, c.ph, p, ns, a, b, cc,
                       dt_host, zseg);
  return hipGetLastError();
}

}  // namespace mhd
