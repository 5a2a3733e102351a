// mhd_kernels.hip -- gfx950 kernels of the explicit MHD step.
//
// stage_kernel: one SSP-RK stage (Sect. 2.9) fused into one launch.  A block
// owns a 14 x 14 column tile of the x-y plane and a segment of z planes; its
// 16 x 16 threads hold one cell column each (the outer ring is the halo of
// the three-cell reconstruction stencil, plus 64 ring cells two columns out
// that only feed the x/y stencils).  The block marches up the segment; per
// plane k it
//   P1  converts plane k+2 to primitive deviations (EOS included) and stages
//       it in LDS (two plane buffers), reconstructs cell k+1 of its own
//       column along z and solves the z-face k+1/2, and reconstructs cell
//       k+1 along x and y from the staged plane (one slope per cell and
//       direction; the upper x value reaches the next lane by a shuffle,
//       the upper y value goes through LDS),
//   P2  solves the Riemann problems of the x- and y-faces of plane k+1,
//   P3  updates the cells of plane k, accumulates the x/y flux divergence of
//       plane k+1 and computes the Contact-CT edge EMFs E_z(k+1), E_x and
//       E_y(k+1/2),
//   P4  updates the faces B_x(k) and B_y(k); B_z(k+1/2), which needs the
//       E_x(k+1/2) of the row above from P3, is updated in the next plane
//       after its first barrier (two barriers per plane, after P1 and P2).
// Neighbour exchanges inside a 16-lane row use lane shuffles; exchanges
// across rows use small LDS arrays.  Fluxes and EMFs on tile borders are
// recomputed by both neighbouring blocks from identical inputs with the
// same code, so every face and edge value is single-valued (div B stays at
// round-off) without atomics or a global EMF array.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {

// Row neighbours inside a 16-lane DPP row (one tile row): row_shr:1 reads
// lane-1, row_shl:1 reads lane+1; the lane at the row edge gets 0 (its
// result is never used).  Must be called with all lanes active.
__device__ __forceinline__ int dpp_shr1(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x111, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_shl1(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x101, 0xf, 0xf, true);
}
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(dpp_shr1(__float_as_int(v)));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(dpp_shl1(__float_as_int(v)));
}
__device__ __forceinline__ double from_left(double v) {
  const int lo = dpp_shr1(__double2loint(v)), hi = dpp_shr1(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
  const int lo = dpp_shl1(__double2loint(v)), hi = dpp_shl1(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// z plane q -> stored plane and mirror flag (reflecting walls)
__device__ __forceinline__ int zsource(const Phys &ph, int q, int &mirror) {
  mirror = 0;
  if (q >= 0 && q < ph.nz) return q;
  if (!ph.reflect) return wrapi(q, ph.nz);
  mirror = 1;
  return q < 0 ? -1 - q : 2 * ph.nz - 1 - q;
}
// z face index f (0..nz for walls) -> stored face
__device__ __forceinline__ int zface(const Phys &ph, int f) {
  return ph.reflect ? f : wrapi(f, ph.nz);
}

struct CellLoad {
  double u[5];
  double b[3];
  double bxl, byl;  // lower x / y faces of the cell (normal fields)
  double tg;
};

// Element access through a plane's address and a lane's column.  The plane
// address (array + field + plane) must be the same for every lane of the
// wave: it is held in scalar registers (the asm's "s" constraint; a base
// the compiler holds in vector registers fails the build with an illegal
// vector-to-scalar copy instead of being narrowed to one lane), and the
// column is a 32-bit byte offset (planes stay below 4 GiB, checked at
// grid creation), so the access takes the scalar-base form of the global
// load and store and costs the vector unit no 64-bit address arithmetic.
// The empty asm statements keep the compiler from folding the scalar base
// into a per-lane address; lane_off re-states a column offset in the basic
// block of its accesses, since the compiler chooses the address form block
// by block.
__device__ __forceinline__ uint32_t lane_off(uint32_t o) {
  asm("" : "+v"(o));
  return o;
}
template <typename T>
__device__ __forceinline__ T plane_ld(const T *base, uint32_t off) {
  using G = const __attribute__((address_space(1))) char;
  using GT = const __attribute__((address_space(1))) T;
  G *b = (G *)base;
  asm("" : "+s"(b));
  return *(GT *)(b + off);
}
template <typename T>
__device__ __forceinline__ void plane_st(T *base, uint32_t off, T v) {
  using G = __attribute__((address_space(1))) char;
  using GT = __attribute__((address_space(1))) T;
  G *b = (G *)base;
  asm("" : "+s"(b));
  *(GT *)(b + off) = v;
}

// byte offsets of a lane's column and of its +x and +y neighbours in a plane
struct ColOff {
  uint32_t c, xp, yp;
};
__device__ __forceinline__ ColOff col_off(const Phys &ph, int gi, int gip, int gj, int gjp) {
  return {(uint32_t)(((size_t)gj * ph.nx + gi) * 8), (uint32_t)(((size_t)gj * ph.nx + gip) * 8),
          (uint32_t)(((size_t)gjp * ph.nx + gi) * 8)};
}

__device__ __forceinline__ void load_cell(const Phys &ph, const StagePtrs &p, ColOff co,
                                          int kk, int mirror, CellLoad &c) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const size_t pk = (size_t)kk * plane;
  const int kp = ph.reflect ? kk + 1 : wrapi(kk + 1, ph.nz);
  const uint32_t o = lane_off(co.c), ox = lane_off(co.xp), oy = lane_off(co.yp);
#pragma unroll
  for (int f = 0; f < 5; ++f) c.u[f] = plane_ld(p.Us + f * n + pk, o);
  c.bxl = plane_ld(p.Bxs + pk, o);
  c.byl = plane_ld(p.Bys + pk, o);
  const double bxr = plane_ld(p.Bxs + pk, ox);
  const double byr = plane_ld(p.Bys + pk, oy);
  const double bzl = plane_ld(p.Bzs + pk, o);
  const double bzr = plane_ld(p.Bzs + (size_t)kp * plane, o);
  c.b[0] = 0.5 * (c.bxl + bxr);
  c.b[1] = 0.5 * (c.byl + byr);
  c.b[2] = 0.5 * (bzl + bzr);
  c.tg = p.Tin ? plane_ld(p.Tin + pk, lane_off(co.c)) : 0.0;
  (void)mirror;
}

template <typename R, bool GR>
struct Cfg {
  static constexpr int NF = GR ? 10 : 8;  // cell fields kept per cell
};

// primitive deviations of one cell, as R, with the mirror image applied
template <typename R, bool GR>
__device__ __forceinline__ void prim_cell(const Phys &ph, const CellLoad &c,
                                          const double bg[4], int mirror, R *w,
                                          PrimOut &o, int maxit = -1) {
  cons2prim<GR>(ph, c.u, c.b, c.tg, bg, o, maxit);
  constexpr int NF = Cfg<R, GR>::NF;
#pragma unroll
  for (int f = 0; f < NF; ++f) w[f] = (R)o.w[f];
  if (mirror) {
    w[Q_VZ] = -w[Q_VZ];
    w[Q_BZ] = -w[Q_BZ];
  }
}

// Number of reconstructed fields per face: rho, v_n, v_t1, v_t2, P, B_t1, B_t2
// (+ gamma_e, gamma_c for the gas+radiation EOS).
template <bool GR>
struct NFS_ {
  static constexpr int v = GR ? 9 : 7;
};

// Reconstruction of one cell along `axis` (0 x, 1 y, 2 z) from its two
// neighbours (Sect. 2.5): the cell's lower-face value lo (R state of face
// i-1/2) and upper-face value hi (L state of face i+1/2), in the face frame
// of the axis (n = axis, t1 = axis+1, t2 = axis+2).  Van Leer: limited
// linear slope; PPH: the unlimited parabola whose averages over the three
// cells are the cell values, lo = (2 m + 5 c - p)/6, hi = (-m + 5 c + 2 p)/6.
template <typename R, bool GR>
__device__ __forceinline__ void recon_cell(int axis, const R *m, const R *c,
                                           const R *p, Side<R> &lo, Side<R> &hi,
                                           bool pph) {
  const int vn = Q_VX + axis, v1 = Q_VX + (axis + 1) % 3, v2 = Q_VX + (axis + 2) % 3;
  const int b1 = Q_BX + (axis + 1) % 3, b2 = Q_BX + (axis + 2) % 3;
  auto rec_vl = [&](int f, R &l, R &h) {
    const R s = R(0.5) * vanleer<R>(c[f] - m[f], p[f] - c[f]);
    l = c[f] - s;
    h = c[f] + s;
  };
  auto rec_pph = [&](int f, R &l, R &h) {
    const R sixth = R(1.0 / 6.0);
    l = (R(2) * m[f] + R(5) * c[f] - p[f]) * sixth;
    h = (R(5) * c[f] - m[f] + R(2) * p[f]) * sixth;
  };
  // one uniform branch per cell and axis, not per field
  auto all = [&](auto rec) {
    rec(Q_RHO, lo.drho, hi.drho);
    rec(vn, lo.vn, hi.vn);
    rec(v1, lo.v1, hi.v1);
    rec(v2, lo.v2, hi.v2);
    rec(Q_P, lo.dp, hi.dp);
    rec(b1, lo.b1, hi.b1);
    rec(b2, lo.b2, hi.b2);
    if (GR) {
      rec(Q_GE, lo.dge, hi.dge);
      rec(Q_GC, lo.dgc, hi.dgc);
    } else {
      lo.dge = hi.dge = lo.dgc = hi.dgc = R(0);
    }
  };
  if (pph)
    all(rec_pph);
  else
    all(rec_vl);
}

template <typename R>
__device__ __forceinline__ Side<R> side_from_left(const Side<R> &s) {
  Side<R> o;
  o.drho = from_left(s.drho);
  o.vn = from_left(s.vn);
  o.v1 = from_left(s.v1);
  o.v2 = from_left(s.v2);
  o.dp = from_left(s.dp);
  o.b1 = from_left(s.b1);
  o.b2 = from_left(s.b2);
  o.dge = from_left(s.dge);
  o.dgc = from_left(s.dgc);
  return o;
}

template <typename R, bool GR>
__device__ __forceinline__ void side_store(R (*buf)[NTHREADS], int t, const Side<R> &s) {
  buf[0][t] = s.drho;
  buf[1][t] = s.vn;
  buf[2][t] = s.v1;
  buf[3][t] = s.v2;
  buf[4][t] = s.dp;
  buf[5][t] = s.b1;
  buf[6][t] = s.b2;
  if (GR) {
    buf[7][t] = s.dge;
    buf[8][t] = s.dgc;
  }
}

template <typename R, bool GR>
__device__ __forceinline__ Side<R> side_load(R (*buf)[NTHREADS], int t) {
  Side<R> s;
  s.drho = buf[0][t];
  s.vn = buf[1][t];
  s.v1 = buf[2][t];
  s.v2 = buf[3][t];
  s.dp = buf[4][t];
  s.b1 = buf[5][t];
  s.b2 = buf[6][t];
  if (GR) {
    s.dge = buf[7][t];
    s.dgc = buf[8][t];
  } else {
    s.dge = s.dgc = R(0);
  }
  return s;
}

// face flux -> conserved order (rho, m_x, m_y, m_z, E)
template <typename R>
__device__ __forceinline__ void to_cons(int axis, const R F[7], R out[5]) {
  out[0] = F[0];
  out[1 + axis] = F[1];
  out[1 + (axis + 1) % 3] = F[2];
  out[1 + (axis + 2) % 3] = F[3];
  out[4] = F[4];
}

// Copy the packed guess network into LDS (all threads; caller syncs).
__device__ __forceinline__ void stage_mlp(const void *src, void *dst, int tid, int nthreads) {
  const uint4 *s4 = (const uint4 *)src;
  uint4 *d4 = (uint4 *)dst;
  for (int i = tid; i < (int)(sizeof(MlpLds) / 16); i += nthreads) d4[i] = s4[i];
}

// The arguments of one stage launch, passed as the kernel's only argument,
// so that they start at offset 0 of the kernel-argument segment.
struct StageArgs {
  Phys ph;
  StagePtrs p;
  double ca, cb, cc, dt_host;  // U^(s+1) = cb U^(s) + ca U^n - cc dt (div F - S)(U^(s))
  int zseg;                    // planes per z segment
};

// The stage's arguments read again from the argument segment, as a view
// the compiler cannot hoist (the asm hides that the address is the same
// each time).  Inside the plane loop the kernel keeps more uniform values
// live (pointers, constants, field offsets, branch conditions) than the
// 102 scalar registers hold; the compiler then parks the excess in lanes
// of vector registers and pays one v_readlane per 32-bit word at every
// use.  Taken from this view once per plane, the values are scalar loads
// (through the scalar cache, no vector issue slot) near their use.
__device__ __forceinline__ const StageArgs &stage_args_view() {
  using KA = const __attribute__((address_space(4))) StageArgs;
  KA *a = (KA *)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(a));
  return *(const StageArgs *)a;
}

// XF: the optional features of a stage (forcing modes, shock-flattening
// flags, species mass fluxes); the variant without them carries none of
// their code, pointers or registers.
template <typename R, bool GR, bool XF>
__global__ __launch_bounds__(NTHREADS) void stage_kernel(StageArgs args) {
  const Phys &ph = args.ph;
  const StagePtrs &p = args.p;
  const double cc = args.cc, dt_host = args.dt_host;
  const int zseg = args.zseg;
  static_assert(sizeof(MlpLds) % 16 == 0, "MlpLds is copied in 16-byte words");
  constexpr int NF = Cfg<R, GR>::NF;
  // FP64 runs one wave per SIMD (register-bound): it has the registers to
  // hold the next plane's cell data while it works on the current one
  constexpr bool PREFETCH = sizeof(R) == 8;
  // the ring cells' data too, except in the gas + radiation variant (its
  // Newton iteration leaves the loads time to arrive; 1 % faster without)
  constexpr bool RING_PREFETCH = PREFETCH && !GR;
  constexpr int NS = NFS_<GR>::v;
  constexpr int LW = TT + 2;  // LDS plane edge: columns -2 .. 15
  constexpr int LP = LW * LW;
  __shared__ R sW[2][NF][LP];       // cell planes by parity
  __shared__ R sYR[NS][NTHREADS];   // upper y-face states of plane k+1
  __shared__ R sYF[5][NTHREADS];    // y-face conserved flux
  __shared__ R sXE[2][NTHREADS];    // x-face E_z, mass flux
  __shared__ R sZE[2][NTHREADS];    // z-face E_x, mass flux
  __shared__ R sRX[2][NTHREADS];    // cell reference E_x, planes by parity
  __shared__ R sRZ[NTHREADS];       // cell reference E_z of plane k+1
  __shared__ R sEZ[2][NTHREADS];    // edge E_z, planes by parity
  __shared__ R sEX[NTHREADS];       // edge E_x(k+1/2)
  __shared__ int sFL[NTHREADS];     // flattening flag of cell k+1

  const int tid = threadIdx.x;
  const int tx = tid % TT, ty = tid / TT;
  const int ci = tx - 1, cj = ty - 1;
  // each XCD works through a contiguous run of tiles (x fastest, then y,
  // then z segment), so neighbouring tiles share its L2
  const int ntx = (ph.nx + TB - 1) / TB, nty = (ph.ny + TB - 1) / TB;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int btx = lb % ntx, bty = (lb / ntx) % nty, bsz = lb / (ntx * nty);
  const int X0 = btx * TB, Y0 = bty * TB;
  const int z0 = bsz * zseg;
  const int z1 = min(z0 + zseg, ph.nz);
  const int gx = X0 + ci, gy = Y0 + cj;
  const int gi = wrapi(gx, ph.nx), gip = wrapi(gx + 1, ph.nx);
  const int gj = wrapi(gy, ph.ny), gjp = wrapi(gy + 1, ph.ny);
  const bool owner = ci >= 0 && ci < TB && cj >= 0 && cj < TB && gx < ph.nx && gy < ph.ny;

  // Background profile (and heating) of the planes this block touches,
  // staged once: cell planes q = z0-2 .. z1+1 (mirror / wrap applied) and
  // z faces z0 .. z1.  Uniform per plane, so every read is a broadcast.
  __shared__ double sBc[5][ZSEG_MAX + 4];  // rho, P, gamma_e, gamma_c, heat
  __shared__ double sBf[4][ZSEG_MAX + 1];
  // forcing from Fourier modes: the z basis of the same planes, and this
  // thread's column coefficients (3 components x FZB), as R
  __shared__ double sZB[XF ? FZB : 1][ZSEG_MAX + 4];
  __shared__ R sFC[XF ? 3 * FZB : 1][NTHREADS];
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t colq = (size_t)gj * ph.nx + gi;
  {
    const int nq = z1 - z0 + 4, nf = z1 - z0 + 1;
    for (int i = threadIdx.x; i < 5 * nq; i += NTHREADS) {
      const int f = i / nq, j = i - f * nq;
      int mir;
      const int kk = zsource(ph, z0 - 2 + j, mir);
      sBc[f][j] = f < 4 ? p.bg_cc[f * ph.nz + kk] : (p.heat ? p.heat[kk] : 0.0);
    }
    for (int i = threadIdx.x; i < 4 * nf; i += NTHREADS) {
      const int f = i / nf, j = i - f * nf;
      sBf[f][j] = p.bg_fz[f * ph.nzf + zface(ph, z0 + j)];
    }
    if (XF && p.fcoef) {
      for (int i = threadIdx.x; i < FZB * nq; i += NTHREADS) {
        const int f = i / nq, j = i - f * nq;
        int mir;
        const int kk = zsource(ph, z0 - 2 + j, mir);
        sZB[f][j] = p.fzb[f * ph.nz + kk];
      }
#pragma unroll
      for (int d = 0; d < 3 * FZB; ++d) sFC[d][threadIdx.x] = (R)p.fcoef[d * plane + colq];
    }
  }
  __syncthreads();

  // ring cells two columns outside the tile (x/y stencils only): the first
  // 16 lanes of each wave take one of the four sides, so that every wave
  // carries the same extra work into the first barrier
  const int lane = tid & 63, wv = tid >> 6;
  const bool ring = lane < 16;
  int rci = 0, rcj = 0;
  if (wv == 0) {
    rci = -2; rcj = lane - 1;
  } else if (wv == 1) {
    rci = TT - 1; rcj = lane - 1;
  } else if (wv == 2) {
    rci = lane - 1; rcj = -2;
  } else {
    rci = lane - 1; rcj = TT - 1;
  }
  const int rgi = wrapi(X0 + rci, ph.nx), rgip = wrapi(X0 + rci + 1, ph.nx);
  const int rgj = wrapi(Y0 + rcj, ph.ny), rgjp = wrapi(Y0 + rcj + 1, ph.ny);
  const ColOff cofs = col_off(ph, gi, gip, gj, gjp), rofs = col_off(ph, rgi, rgip, rgj, rgjp);
  const int lw_own = (cj + 2) * LW + (ci + 2);
  const int lw_ring = (rcj + 2) * LW + (rci + 2);
  const int tdn = tid >= TT ? tid - TT : tid;            // (ci, cj-1)
  const int tdl = tid >= TT + 1 ? tid - TT - 1 : tid;    // (ci-1, cj-1)
  const int tup = tid + TT < NTHREADS ? tid + TT : tid;  // (ci, cj+1)

  const double dt = p.dt_dev ? *p.dt_dev : dt_host;
  const double cdt = cc * dt;
  const R gam = (R)ph.gamma, igm1 = (R)ph.igm1;
  const R mcut = (R)ph.mach_cut, imcut = (R)ph.imach_cut;
  const bool pph = ph.recon == MHD_RECON_PPH;

  // own column state carried along z
  R Wc[NF];        // cell k+1
  Side<R> topk{};  // upper z-face state of cell k (L state of face k+1/2)
  R bxf_c = 0, byf_c = 0;  // normal fields on the lower x / y face, plane k+1
  double acc[5] = {0, 0, 0, 0, 0};  // x/y flux divergence of plane k
  R fzp[5] = {0, 0, 0, 0, 0};       // z-face conserved flux at k-1/2
  R ex_prev = 0, ey_prev = 0;       // own edges E_x, E_y at k-1/2
  R ez_cur = 0;                     // own edge E_z at plane k
  double bzf_prev = 0.0, bz0_prev = 0.0;  // B_z^(s), B_z^n of the face k+1/2 of the previous plane
  R xf_ey_prev = 0, xf_m_prev = 0;  // own x-face E_y and mass flux, plane k
  R yf_ex_prev = 0, yf_m_prev = 0;  // own y-face E_x and mass flux, plane k
  R rx_prev = 0, ry_prev = 0;       // own cell reference E_x, E_y, plane k
  // shock-flattening flags of the own column's cells k and k+1 (Sect. 2.7):
  // a flagged cell is reconstructed with van Leer, and every face it
  // touches takes the HLL flux
  int fk = 0, fc = 0;
  unsigned long long nit = 0, nmax = 0, nfb = 0;
  int bad = 0;
#pragma unroll
  for (int f = 0; f < NF; ++f) Wc[f] = R(0);

  CellLoad pc{}, prc{};  // prefetched cell data of the next P1 plane
  if (PREFETCH) {
    int mir0;
    const int k0 = zsource(ph, z0 - 2, mir0);
    load_cell(ph, p, cofs, k0, mir0, pc);
    if (RING_PREFETCH && ring) load_cell(ph, p, rofs, k0, mir0, prc);
  }
  for (int k = z0 - 4; k < z1; ++k) {
    // this plane's view of the arguments (shadows the kernel's own names);
    // FP32 variants only: the FP64 kernel, one wave per SIMD and bound by
    // latency, ran no faster with the scalar loads (the gas+radiation
    // variant 0.7 % slower)
    const StageArgs &A = sizeof(R) == 4 ? stage_args_view() : args;
    const Phys &ph = A.ph;
    const StagePtrs &p = A.p;
    const double ca = A.ca, cb = A.cb;
    const size_t plane = (size_t)ph.nx * ph.ny;
    const size_t ncell = plane * ph.nz;
    // every global value P3 and P4 read, requested together at the top of
    // the plane so that the latency overlaps P1 and P2
    const bool upd = k >= z0 && owner;
    const bool updz = k >= z0 - 1 && k + 1 < z1 && owner && !(ph.reflect && k + 1 == 0);
    const bool base = ca != 0.0;
    double us[5] = {0, 0, 0, 0, 0}, u0[5] = {0, 0, 0, 0, 0};
    double bxs = 0.0, bys = 0.0, bx0 = 0.0, by0 = 0.0, bz0 = 0.0;
    const size_t pqc = (size_t)(k > 0 ? k : 0) * plane;
    const size_t pqf = (size_t)(k + 1 > 0 ? k + 1 : 0) * plane;
    if (upd) {
      const uint32_t o = lane_off(cofs.c);
#pragma unroll
      for (int f = 0; f < 5; ++f) us[f] = plane_ld(p.Us + f * ncell + pqc, o);
      bxs = plane_ld(p.Bxs + pqc, o);
      bys = plane_ld(p.Bys + pqc, o);
    }
    if (upd && base) {
      const uint32_t o = lane_off(cofs.c);
#pragma unroll
      for (int f = 0; f < 5; ++f) u0[f] = plane_ld(p.U0 + f * ncell + pqc, o);
      bx0 = plane_ld(p.Bx0 + pqc, o);
      by0 = plane_ld(p.By0 + pqc, o);
    }
    if (updz && base) bz0 = plane_ld(p.Bz0 + pqf, lane_off(cofs.c));
    // ---------------- P1 ------------------------------------------------
    // primitives of plane k+2 (staged in LDS), z reconstruction of cell
    // k+1 and the z-face k+1/2, x/y reconstruction of cell k+1
    R Wn[NF];
    R bxf_n, byf_n;
    double bzf = 0.0;  // B_z on the z-face k+1/2 (read again by P4)
    R fzc[5] = {0, 0, 0, 0, 0};
    R zf_ey = 0, zf_ex = 0, zf_m = 0;
    Side<R> xl{}, xll{}, yl{};
    R rx = 0, ry = 0, rz = 0;
    int fn = 0;  // flag of cell k+2 (a mirror image carries its source's)
    {
      const int q = k + 2;
      int mir;
      const int kk = zsource(ph, q, mir);
      if (XF && p.flat) fn = plane_ld(p.flat + (size_t)kk * plane, lane_off(cofs.c >> 3));
      R *sWn = &sW[q & 1][0][0];
      CellLoad c, rc;
      if (PREFETCH) {
        // plane q arrived during the previous plane; request plane q+1
        c = pc;
        if (RING_PREFETCH) rc = prc;
        if (k + 1 < z1) {
          int mirn;
          const int kn = zsource(ph, q + 1, mirn);
          load_cell(ph, p, cofs, kn, mirn, pc);
          if (RING_PREFETCH && ring) load_cell(ph, p, rofs, kn, mirn, prc);
        }
      } else {
        load_cell(ph, p, cofs, kk, mir, c);
      }
      const int maxit = p.newton_cap;
      const int jq = q - (z0 - 2);
      const double bgq[4] = {sBc[0][jq], sBc[1][jq], sBc[2][jq], sBc[3][jq]};
      {
        PrimOut o;
        prim_cell<R, GR>(ph, c, bgq, mir, Wn, o, maxit);
        bxf_n = (R)c.bxl;
        byf_n = (R)c.byl;
        if (GR) {
          if (owner && q >= z0 && q < z1) {
            if (p.Tout) plane_st(p.Tout + (size_t)kk * plane, lane_off(cofs.c), o.T);
            nit += o.iters;
            nmax = o.iters > nmax ? o.iters : nmax;
            nfb += o.fallback;
          }
        }
        bad |= o.bad;
      }
      if (ring) {
        if (!RING_PREFETCH) load_cell(ph, p, rofs, kk, mir, rc);
        PrimOut ro;
        R Wr[NF];
        prim_cell<R, GR>(ph, rc, bgq, mir, Wr, ro, maxit);
        bad |= ro.bad;
#pragma unroll
        for (int f = 0; f < NF; ++f) sWn[f * LP + lw_ring] = Wr[f];
      }
      // own cell k sits in the slot the new plane goes to; only this thread
      // reads or writes that slot
      R Wm[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        Wm[f] = sWn[f * LP + lw_own];
        sWn[f * LP + lw_own] = Wn[f];
      }
      if (k >= z0 - 2) {
        Side<R> botn, topn;
        const bool pphc = pph && !(XF && fc);
        recon_cell<R, GR>(2, Wm, Wc, Wn, botn, topn, pphc);
        if (k >= z0 - 1) {
          const int fzi = zface(ph, k + 1);
          FaceBg<R> bgf;
          const int jf = k + 1 - z0;
          bgf.rho = (R)sBf[0][jf];
          bgf.p = (R)sBf[1][jf];
          bgf.ge = (R)sBf[2][jf];
          bgf.gc = (R)sBf[3][jf];
          bzf = plane_ld(p.Bzs + (size_t)fzi * plane, lane_off(cofs.c));
          const R bzn = (R)bzf;
          R fz[7];
          face_flux<R, GR>(XF && (fk | fc) != 0, topk, botn, bzn, bgf, gam, igm1, ph.xi_mode,
                           mcut, imcut, fz);
          // mass flux for the species: the lower face of cell k+1 (and the
          // top wall), written once, by the block that owns the cell
          const int f = k + 1;
          if (XF && p.mfz && owner && ((f >= z0 && f < z1) || (ph.reflect && f == ph.nz)))
            plane_st(p.mfz + (size_t)f * plane, lane_off(cofs.c), (double)fz[0]);
          to_cons<R>(2, fz, fzc);
          zf_ey = -fz[5];  // z-face E_y = -F_z[B_x]
          zf_ex = fz[6];   // z-face E_x = +F_z[B_y]
          zf_m = fz[0];
        }
        topk = topn;
        // x/y reconstruction of cell k+1 from the staged plane k+1
        const R *sWc = &sW[(k + 1) & 1][0][0];
        // neighbours at ci-1 >= -2 and cj-1 >= -2 are staged (ring cells
        // included): the halo column ci = -1 supplies the L state of the
        // tile's first x-face
        R a[NF], b[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          a[f] = sWc[f * LP + lw_own - 1];
          b[f] = sWc[f * LP + lw_own + 1];
        }
        Side<R> xh;
        recon_cell<R, GR>(0, a, Wc, b, xl, xh, pphc);
        xll = side_from_left<R>(xh);  // L state of the x-face ci-1/2
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          a[f] = sWc[f * LP + lw_own - LW];
          b[f] = sWc[f * LP + lw_own + LW];
        }
        Side<R> yh;
        recon_cell<R, GR>(1, a, Wc, b, yl, yh, pphc);
        side_store<R, GR>(sYR, tid, yh);
        if (XF) sFL[tid] = fc;
        // cell reference EMF -(v x B) of plane k+1
        rx = -(Wc[Q_VY] * Wc[Q_BZ] - Wc[Q_VZ] * Wc[Q_BY]);
        ry = -(Wc[Q_VZ] * Wc[Q_BX] - Wc[Q_VX] * Wc[Q_BZ]);
        rz = -(Wc[Q_VX] * Wc[Q_BY] - Wc[Q_VY] * Wc[Q_BX]);
      }
    }
    __syncthreads();

    // ---------------- B_z(k-1/2), the previous plane's z-face ------------
    // its E_x neighbour (the row above) comes from that plane's P3, visible
    // since the barrier above; the next write of sEX follows the barrier
    // after P2
    {
      const R ey_r = from_right(ey_prev);
      const bool updz_prev = k - 1 >= z0 - 1 && k < z1 && owner && !(ph.reflect && k == 0);
      if (updz_prev) {
        const double ex_u = (double)sEX[tup];
        const double rbz = ((double)ey_r - (double)ey_prev) * ph.idx -
                           (ex_u - (double)ex_prev) * ph.idy;
        plane_st(p.Bzo + pqc, lane_off(cofs.c), cb * bzf_prev - cdt * rbz + ca * bz0_prev);
      }
    }

    // ---------------- P2: x- and y-faces of plane k+1 --------------------
    R fx[7], fy[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) fx[c] = fy[c] = R(0);
    if (k >= z0 - 2) {
      const int jc = k + 1 - (z0 - 2);
      FaceBg<R> bgc;
      bgc.rho = (R)sBc[0][jc];
      bgc.p = (R)sBc[1][jc];
      bgc.ge = (R)sBc[2][jc];
      bgc.gc = (R)sBc[3][jc];
      const bool hx = XF && (fc | dpp_shr1(fc)) != 0;  // cells ci-1 and ci
      face_flux<R, GR>(hx, xll, xl, bxf_c, bgc, gam, igm1, ph.xi_mode, mcut, imcut, fx);
      const Side<R> yll = side_load<R, GR>(sYR, tdn);
      const bool hy = XF && (fc | sFL[tdn]) != 0;  // cells cj-1 and cj
      face_flux<R, GR>(hy, yll, yl, byf_c, bgc, gam, igm1, ph.xi_mode, mcut, imcut, fy);
      R fyc[5];
      to_cons<R>(1, fy, fyc);
#pragma unroll
      for (int f = 0; f < 5; ++f) sYF[f][tid] = fyc[f];
      // mass fluxes for the species: the lower x and y faces of the owned
      // cells of plane k+1
      if (XF && p.mfx && owner && k + 1 >= z0 && k + 1 < z1) {
        const size_t pf = (size_t)(k + 1) * plane;
        const uint32_t o = lane_off(cofs.c);
        plane_st(p.mfx + pf, o, (double)fx[0]);
        plane_st(p.mfy + pf, o, (double)fy[0]);
      }
      sXE[0][tid] = -fx[5];  // x-face E_z = -F_x[B_y]
      sXE[1][tid] = fx[0];
      sZE[0][tid] = zf_ex;
      sZE[1][tid] = zf_m;
      sRX[(k + 1) & 1][tid] = rx;
      sRZ[tid] = rz;
    }
    __syncthreads();

    // ---------------- P3: cells of plane k, divergence, edge EMFs -------
    R fxc[5];
    to_cons<R>(0, fx, fxc);
    R fxr[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) fxr[f] = from_right(fxc[f]);
    // neighbour data at ci-1 (same row)
    const R yf_ez_l = from_left(fy[6]);  // y-face E_z = +F_y[B_x]
    const R yf_m_l = from_left(fy[0]);
    const R rz_l = from_left(rz);
    const R zf_ey_l = from_left(zf_ey);
    const R zf_m_l = from_left(zf_m);
    const R ry_l = from_left(ry);
    const R ry_prev_l = from_left(ry_prev);
    R ex_new = 0, ey_new = 0, ez_new = 0;
    if (k >= z0 - 1) {
      // cells of plane k
      if (upd) {
        double r[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) r[f] = acc[f] + ((double)fzc[f] - (double)fzp[f]) * ph.idz;
        // sources S - S_hat: gravity on the density deviation, rho g.v,
        // heating, forcing (Sect. 2.1, eq. wb2)
        const int jk = k - (z0 - 2);
        double s1 = 0.0, s2 = 0.0, s3 = (us[0] - sBc[0][jk]) * ph.gz;
        double s4 = us[3] * ph.gz + sBc[4][jk];
        if (XF && p.fcoef) {
          // the forcing of this cell from its column's coefficients
          double fo[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double f = 0.0;
#pragma unroll
            for (int d = 0; d < FZB; ++d) f += (double)sFC[c * FZB + d][tid] * sZB[d][jk];
            fo[c] = f;
          }
          s1 += us[0] * fo[0];
          s2 += us[0] * fo[1];
          s3 += us[0] * fo[2];
          s4 += us[1] * fo[0] + us[2] * fo[1] + us[3] * fo[2];
        }
        r[1] -= s1;
        r[2] -= s2;
        r[3] -= s3;
        r[4] -= s4;
        {
          const uint32_t o = lane_off(cofs.c);
#pragma unroll
          for (int f = 0; f < 5; ++f)
            plane_st(p.Uo + f * ncell + pqc, o, cb * us[f] - cdt * r[f] + ca * u0[f]);
        }
      }
      // x/y divergence of plane k+1
      R fyc[5];
      to_cons<R>(1, fy, fyc);
#pragma unroll
      for (int f = 0; f < 5; ++f)
        acc[f] = ((double)fxr[f] - (double)fxc[f]) * ph.idx +
                 ((double)sYF[f][tup] - (double)fyc[f]) * ph.idy;
      // E_z at (ci-1/2, cj-1/2, k+1): a = x, b = y
      ez_new = ct_edge<R>(-fx[5], sXE[0][tdn], fy[6], yf_ez_l, rz, rz_l, sRZ[tdn],
                          sRZ[tdl], fx[0], sXE[1][tdn], fy[0], yf_m_l);
      // E_x at (ci, cj-1/2, k+1/2): a = y (y-faces at planes k+1, k),
      // b = z (z-faces at cj, cj-1)
      const int s1 = (k + 1) & 1, s0 = k & 1;
      ex_new = ct_edge<R>(-fy[5], yf_ex_prev, zf_ex, sZE[0][tdn], rx, sRX[s1][tdn], rx_prev,
                          sRX[s0][tdn], fy[0], yf_m_prev, zf_m, sZE[1][tdn]);
      // E_y at (ci-1/2, cj, k+1/2): a = z (z-faces at ci, ci-1), b = x
      // (x-faces at planes k+1, k)
      ey_new = ct_edge<R>(zf_ey, zf_ey_l, fx[6], xf_ey_prev, ry, ry_prev, ry_l, ry_prev_l,
                          zf_m, zf_m_l, fx[0], xf_m_prev);
      // a reflecting wall carries no tangential EMF
      if (ph.reflect && (k + 1 == 0 || k + 1 == ph.nz)) {
        ex_new = R(0);
        ey_new = R(0);
      }
      sEZ[(k + 1) & 1][tid] = ez_new;
      sEX[tid] = ex_new;
    }

    // ---------------- P4: faces B_x(k), B_y(k) ---------------------------
    // E_z of the row above at plane k comes from the previous plane's P3
    const R ez_r = from_right(ez_cur);
    if (upd) {
      const double ez_u = (double)sEZ[k & 1][tup];
      const double rbx = (ez_u - (double)ez_cur) * ph.idy -
                         ((double)ey_new - (double)ey_prev) * ph.idz;
      const double rby = ((double)ex_new - (double)ex_prev) * ph.idz -
                         ((double)ez_r - (double)ez_cur) * ph.idx;
      const uint32_t o = lane_off(cofs.c);
      plane_st(p.Bxo + pqc, o, cb * bxs - cdt * rbx + ca * bx0);
      plane_st(p.Byo + pqc, o, cb * bys - cdt * rby + ca * by0);
    }
    bzf_prev = bzf;
    bz0_prev = bz0;

    // ---------------- shift the pipeline --------------------------------
    ez_cur = ez_new;
    ex_prev = ex_new;
    ey_prev = ey_new;
#pragma unroll
    for (int f = 0; f < 5; ++f) fzp[f] = fzc[f];
    xf_ey_prev = fx[6];
    xf_m_prev = fx[0];
    yf_ex_prev = -fy[5];
    yf_m_prev = fy[0];
    rx_prev = rx;
    ry_prev = ry;
#pragma unroll
    for (int f = 0; f < NF; ++f) Wc[f] = Wn[f];
    bxf_c = bxf_n;
    byf_c = byf_n;
    fk = fc;
    fc = fn;
  }
  if (bad) atomicOr(p.flags, bad);
  if (GR) {
    // block totals of the Newton statistics
    __shared__ unsigned long long s_it[NTHREADS / 64], s_fb[NTHREADS / 64], s_mx[NTHREADS / 64];
    unsigned long long a = nit, f = nfb, m = nmax;
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      f += __shfl_xor(f, o);
      unsigned long long mo = __shfl_xor(m, o);
      m = mo > m ? mo : m;
    }
    if ((tid & 63) == 0) {
      s_it[tid >> 6] = a;
      s_fb[tid >> 6] = f;
      s_mx[tid >> 6] = m;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long A = 0, Fb = 0, M = 0;
      for (int w = 0; w < NTHREADS / 64; ++w) {
        A += s_it[w];
        Fb += s_fb[w];
        M = s_mx[w] > M ? s_mx[w] : M;
      }
      atomicAdd(&p.newton_stats[0], A);
      atomicMax(&p.newton_stats[1], M);
      atomicAdd(&p.newton_stats[2], Fb);
    }
  }
}

size_t mlp_bytes() { return sizeof(MlpLds); }

template <typename R, bool GR>
static void launch_stage_g(const Ctx &c, const StagePtrs &p, double a, double b, double cc,
                           double dt_host, dim3 grid) {
  dim3 block(NTHREADS);
  if (p.fcoef || p.flat || p.mfx || p.mfy || p.mfz)
    hipLaunchKernelGGL((stage_kernel<R, GR, true>), grid, block, 0, c.stream,
                       StageArgs{c.ph, p, a, b, cc, dt_host, c.zseg});
  else
    hipLaunchKernelGGL((stage_kernel<R, GR, false>), grid, block, 0, c.stream,
                       StageArgs{c.ph, p, a, b, cc, dt_host, c.zseg});
}

template <typename R>
static void launch_stage_t(const Ctx &c, const StagePtrs &p, double a, double b, double cc,
                           double dt_host, dim3 grid) {
  if (!c.ph.gasrad)
    launch_stage_g<R, false>(c, p, a, b, cc, dt_host, grid);
  else
    launch_stage_g<R, true>(c, p, a, b, cc, dt_host, grid);
}

// the variant the context's stages run (occupancy for the segment length;
// forcing modes set later only change the variant, not the result)
template <typename R>
static const void *stage_fn(const Ctx &c) {
  const bool xf = c.d.flatten || c.d.nspecies > 0;
  if (!c.ph.gasrad)
    return xf ? reinterpret_cast<const void *>(&stage_kernel<R, false, true>)
              : reinterpret_cast<const void *>(&stage_kernel<R, false, false>);
  return xf ? reinterpret_cast<const void *>(&stage_kernel<R, true, true>)
            : reinterpret_cast<const void *>(&stage_kernel<R, true, false>);
}

int stage_blocks_per_cu(const Ctx &c) {
  const void *f = c.d.precision == MHD_PREC_SPLIT ? stage_fn<float>(c) : stage_fn<double>(c);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, NTHREADS, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

hipError_t launch_stage(const Ctx &c, const StagePtrs &p, double a, double b,
                        double cc, double dt_host) {
  const Phys &ph = c.ph;
  const int nblk = ((ph.nx + TB - 1) / TB) * ((ph.ny + TB - 1) / TB) * ((ph.nz + c.zseg - 1) / c.zseg);
  dim3 grid(nblk);
  if (c.d.precision == MHD_PREC_SPLIT)
    launch_stage_t<float>(c, p, a, b, cc, dt_host, grid);
  else
    launch_stage_t<double>(c, p, a, b, cc, dt_host, grid);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CFL time step (eq. cfl): per-cell signal speed, block max, final max
// ---------------------------------------------------------------------------

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = CFL_MAX_BLOCKS;

template <bool GR, bool ML>
// Three waves per SIMD at least: the variant with the learned guess would
// otherwise take 181 registers (two waves) and wait on memory; at 168 it
// spills five registers and runs 8 % faster (the other variants use 66).
__global__ __launch_bounds__(RED_THREADS) __attribute__((amdgpu_waves_per_eu(3))) void
signal_speed_kernel(
    Phys ph, const double *__restrict__ U, const double *__restrict__ Bx,
    const double *__restrict__ By, const double *__restrict__ Bz,
    const double *__restrict__ T, const void *mlp, double *__restrict__ partial,
    int *flags, double *__restrict__ Tout, double *__restrict__ Pout) {
  __shared__ __attribute__((aligned(16))) char sMlpRaw[ML ? sizeof(MlpLds) : 16];
  const MlpLds &sMlp = *reinterpret_cast<const MlpLds *>(sMlpRaw);
  if (ML) {
    stage_mlp(mlp, sMlpRaw, threadIdx.x, RED_THREADS);
    __syncthreads();
  }
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const int lane = threadIdx.x & 63;
  double smax = 0.0;
  int bad = 0;
  // uniform trip count: lanes past the end redo the last cell and drop it
  for (size_t base = (size_t)blockIdx.x * blockDim.x; base < n;
       base += (size_t)gridDim.x * blockDim.x) {
    const bool valid = base + threadIdx.x < n;
    const size_t q = valid ? base + threadIdx.x : n - 1;
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
    const double zero[4] = {0, 0, 0, 0};
    double tg = (GR && !ML && T) ? T[q] : 0.0;
    if (ML) {
      float x0, x1;
      mlp_inputs(ph, u[0], specific_eint(u, b), x0, x1);
      tg = mlp_guess_wave(ph, sMlp, x0, x1, lane);
    }
    PrimOut o;
    cons2prim<GR>(ph, u, b, tg, zero, o, ML ? ph.newton_maxit_mlp : ph.newton_maxit);
    if (!valid) continue;
    bad |= o.bad;
    // the converged temperature is the best guess the next stage can get
    if (GR && Tout) Tout[q] = o.T;
    if (Pout) Pout[q] = o.w[Q_P];  // thermal pressure for the flattening detector
    const double rho = u[0];
    const double P = o.w[Q_P];
    const double a2 = o.w[Q_GC] * P / rho;
    const double b2 = (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) / rho;
    const double v[3] = {o.w[Q_VX], o.w[Q_VY], o.w[Q_VZ]};
    const double ids[3] = {ph.idx, ph.idy, ph.idz};
    double sum = 0.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (!ph.dims_active[s]) continue;
      const double bs2 = b[s] * b[s] / rho;
      double disc = (a2 + b2) * (a2 + b2) - 4.0 * a2 * bs2;
      disc = disc > 0.0 ? disc : 0.0;
      const double cf = sqrt(0.5 * ((a2 + b2) + sqrt(disc)));
      sum += (fabs(v[s]) + cf) * ids[s];
    }
    smax = sum > smax ? sum : smax;
    if (!(sum < INFINITY)) bad |= 1;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double t = __shfl_xor(smax, o);
    smax = t > smax ? t : smax;
  }
  __shared__ double sm[RED_THREADS / 64];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = smax;
  if (bad) atomicOr(flags, bad);
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) m = sm[w] > m ? sm[w] : m;
    partial[blockIdx.x] = m;
  }
}

__global__ void finish_dt_kernel(const double *__restrict__ partial, int nb,
                                 double cfl, double *dt_out, double *smax_out) {
  __shared__ double sm[RED_THREADS];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = partial[i] > m ? partial[i] : m;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = sm[threadIdx.x + s] > sm[threadIdx.x] ? sm[threadIdx.x + s] : sm[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *smax_out = sm[0];
    *dt_out = cfl / sm[0];
  }
}

int cfl_partial_blocks(size_t ncell) {
  const size_t nb = (ncell + RED_THREADS - 1) / RED_THREADS;
  return (int)(nb < (size_t)RED_BLOCKS ? nb : (size_t)RED_BLOCKS);
}

hipError_t launch_signal_speed_raw(const Phys &ph, hipStream_t stream, bool learned,
                                   const double *U, const double *Bx, const double *By,
                                   const double *Bz, const double *T, const void *mlp,
                                   double *partial, int *flags, double cfl, double *dt_dev,
                                   double *smax_out, double *Tout, double *Pout) {
  const int nb = cfl_partial_blocks((size_t)ph.nx * ph.ny * ph.nz);
  if (!ph.gasrad)
    hipLaunchKernelGGL((signal_speed_kernel<false, false>), dim3(nb), dim3(RED_THREADS), 0,
                       stream, ph, U, Bx, By, Bz, T, mlp, partial, flags, nullptr, Pout);
  else if (learned)
    hipLaunchKernelGGL((signal_speed_kernel<true, true>), dim3(nb), dim3(RED_THREADS), 0,
                       stream, ph, U, Bx, By, Bz, T, mlp, partial, flags, Tout, Pout);
  else
    hipLaunchKernelGGL((signal_speed_kernel<true, false>), dim3(nb), dim3(RED_THREADS), 0,
                       stream, ph, U, Bx, By, Bz, T, mlp, partial, flags, Tout, Pout);
  hipLaunchKernelGGL(finish_dt_kernel, dim3(1), dim3(RED_THREADS), 0, stream, partial, nb, cfl,
                     dt_dev, smax_out);
  return hipGetLastError();
}

hipError_t launch_signal_speed(const Ctx &c, const double *U, const double *Bx,
                               const double *By, const double *Bz,
                               const double *T, double cfl, double *dt_dev, double *Tout,
                               double *Pout) {
  return launch_signal_speed_raw(c.ph, c.stream, c.d.eos_guess == MHD_GUESS_MLP, U, Bx, By, Bz,
                                 T, c.mlp, c.red, c.flags, cfl, dt_dev, c.red + RED_BLOCKS, Tout,
                                 Pout);
}

// ---------------------------------------------------------------------------
// initial temperature (bracketed solve) for the previous-T guess
// ---------------------------------------------------------------------------

// T of every cell: Newton from Tg when given, else the bracketed solve
__global__ void init_temperature_kernel(Phys ph, const double *__restrict__ U,
                                        const double *__restrict__ Bx,
                                        const double *__restrict__ By,
                                        const double *__restrict__ Bz,
                                        const double *__restrict__ Tg,
                                        double *__restrict__ T, int *flags) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const int ip = i + 1 == ph.nx ? 0 : i + 1;
    const int jp = j + 1 == ph.ny ? 0 : j + 1;
    const int kp = ph.reflect ? k + 1 : (k + 1 == ph.nz ? 0 : k + 1);
    double u[5], b[3];
    for (int f = 0; f < 5; ++f) u[f] = U[f * n + q];
    b[0] = 0.5 * (Bx[q] + Bx[q - i + ip]);
    b[1] = 0.5 * (By[q] + By[q + (size_t)(jp - j) * ph.nx]);
    b[2] = 0.5 * (Bz[q] + Bz[(size_t)kp * plane + (q - (size_t)k * plane)]);
    const double zero[4] = {0, 0, 0, 0};
    PrimOut o;
    cons2prim<true>(ph, u, b, Tg ? Tg[q] : NAN, zero, o);
    if (o.bad) atomicOr(flags, o.bad);
    T[q] = o.T;
  }
}

hipError_t launch_init_temperature(const Ctx &c, const double *U,
                                   const double *Bx, const double *By,
                                   const double *Bz, const double *Tg, double *T) {
  int nb = (int)((c.ncell + 255) / 256);
  nb = nb < 4096 ? nb : 4096;
  hipLaunchKernelGGL(init_temperature_kernel, dim3(nb), dim3(256), 0, c.stream, c.ph, U, Bx, By,
                     Bz, Tg, T, c.flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// learned initial guess of every cell of a state (before each stage in the
// learned mode): the stage kernel reads it as its temperature guess
// ---------------------------------------------------------------------------

// With polish the guess is polished by FP64 Newton right here (at most
// newton_maxit_mlp steps, then the bracketed solve) and the converged
// temperature is stored in its place, so the stage's own Newton starts
// converged: the iterations run in this small kernel at full occupancy
// instead of in the register-bound stage.  Their statistics go to stats
// (nullable).  With P != nullptr (shock flattening) the thermal pressure
// the detector needs is stored as well.
__global__ __launch_bounds__(256) void mlp_guess_kernel(Phys ph, const double *__restrict__ U,
                                                        const double *__restrict__ Bx,
                                                        const double *__restrict__ By,
                                                        const double *__restrict__ Bz,
                                                        const void *mlp,
                                                        double *__restrict__ Tg,
                                                        double *__restrict__ P, int *flags,
                                                        int polish,
                                                        unsigned long long *stats) {
  __shared__ __attribute__((aligned(16))) char sMlpRaw[sizeof(MlpLds)];
  const MlpLds &sMlp = *reinterpret_cast<const MlpLds *>(sMlpRaw);
  stage_mlp(mlp, sMlpRaw, threadIdx.x, 256);
  __syncthreads();
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const int lane = threadIdx.x & 63;
  // every lane of a wave runs the matrix passes; lanes past the end repeat
  // the last cell and store nothing
  // cell data of one cell: U and the six faces (read at the top of each
  // pass: without a prefetch of the next cell the kernel fits 156 registers
  // and three waves per SIMD, which hide the latency better)
  auto fetch = [&](size_t q, double u[5], double f[6]) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const int ip = i + 1 == ph.nx ? 0 : i + 1;
    const int jp = j + 1 == ph.ny ? 0 : j + 1;
    const int kp = ph.reflect ? k + 1 : (k + 1 == ph.nz ? 0 : k + 1);
#pragma unroll
    for (int c = 0; c < 5; ++c) u[c] = U[c * n + q];
    f[0] = Bx[q];
    f[1] = Bx[q - i + ip];
    f[2] = By[q];
    f[3] = By[q + (size_t)(jp - j) * ph.nx];
    f[4] = Bz[q];
    f[5] = Bz[(size_t)kp * plane + (q - (size_t)k * plane)];
  };
  const size_t stride = (size_t)gridDim.x * 256;
  size_t base = (size_t)blockIdx.x * 256;
  unsigned long long nit = 0, nmax = 0, nfb = 0;
  for (; base < n; base += stride) {
    const bool valid = base + threadIdx.x < n;
    const size_t q = valid ? base + threadIdx.x : n - 1;
    double u[5], b[3], fn[6];
    fetch(q, u, fn);
    b[0] = 0.5 * (fn[0] + fn[1]);
    b[1] = 0.5 * (fn[2] + fn[3]);
    b[2] = 0.5 * (fn[4] + fn[5]);
    float x0, x1;
    const double e = specific_eint(u, b);
    mlp_inputs(ph, u[0], e, x0, x1);
    const double t = mlp_guess_wave(ph, sMlp, x0, x1, lane);
    if (!valid) continue;
    if (!polish) {
      Tg[q] = t;
      continue;
    }
    const double zero_bg[4] = {0.0, 0.0, 0.0, 0.0};
    PrimOut o;
    cons2prim<true>(ph, u, b, t, zero_bg, o, ph.newton_maxit_mlp);
    if (o.bad) atomicOr(flags, o.bad);
    nit += o.iters;
    nmax = o.iters > nmax ? o.iters : nmax;
    nfb += o.fallback;
    Tg[q] = o.T;
    if (P) P[q] = o.w[Q_P];  // full pressure: the background passed is zero
  }
  if (stats) {
    // block totals of the Newton statistics
    __shared__ unsigned long long s_it[4], s_fb[4], s_mx[4];
    for (int o = 32; o > 0; o >>= 1) {
      nit += __shfl_xor(nit, o);
      nfb += __shfl_xor(nfb, o);
      const unsigned long long m = __shfl_xor(nmax, o);
      nmax = m > nmax ? m : nmax;
    }
    if (lane == 0) {
      s_it[threadIdx.x >> 6] = nit;
      s_fb[threadIdx.x >> 6] = nfb;
      s_mx[threadIdx.x >> 6] = nmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long a = 0, f = 0, m = 0;
      for (int w = 0; w < 4; ++w) {
        a += s_it[w];
        f += s_fb[w];
        m = s_mx[w] > m ? s_mx[w] : m;
      }
      atomicAdd(&stats[0], a);
      atomicMax(&stats[1], m);
      atomicAdd(&stats[2], f);
    }
  }
}

hipError_t launch_mlp_guess(const Ctx &c, const double *U, const double *Bx, const double *By,
                            const double *Bz, double *Tg, double *P, bool polish,
                            unsigned long long *stats) {
  long long nb = (long long)((c.ncell + 255) / 256);
  nb = nb < 8192 ? nb : 8192;
  hipLaunchKernelGGL(mlp_guess_kernel, dim3((unsigned)nb), dim3(256), 0, c.stream, c.ph, U, Bx,
                     By, Bz, c.mlp, Tg, P, c.flags, polish ? 1 : 0, stats);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batch temperature inversion T(rho, e_int) (EOS microbenchmark and guess
// quality): guess from an array, the learned network or the bracket
// ---------------------------------------------------------------------------

template <bool ML>
__global__ __launch_bounds__(256) void eos_solve_kernel(
    Phys ph, const double *__restrict__ rho, const double *__restrict__ e,
    const double *__restrict__ tguess, long long n, const void *mlp,
    double *__restrict__ T, double *__restrict__ T0, unsigned long long *stats, int *flags) {
  __shared__ __attribute__((aligned(16))) char sMlpRaw[ML ? sizeof(MlpLds) : 16];
  const MlpLds &sMlp = *reinterpret_cast<const MlpLds *>(sMlpRaw);
  if (ML) {
    stage_mlp(mlp, sMlpRaw, threadIdx.x, 256);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  unsigned long long it = 0, mx = 0, fb = 0;
  int bad = 0;
  // the next sample's inputs are requested before this one is solved
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long base = (long long)blockIdx.x * blockDim.x;
  double rn = 0.0, en = 0.0, gn = NAN;
  if (base < n) {
    const long long q0 = base + threadIdx.x < n ? base + threadIdx.x : n - 1;
    rn = rho[q0];
    en = e[q0];
    if (tguess) gn = tguess[q0];
  }
  for (; base < n; base += stride) {
    const bool valid = base + threadIdx.x < n;
    const long long q = valid ? base + threadIdx.x : n - 1;
    const double r = rn, ee = en;
    double g = gn;
    if (base + stride < n) {
      const long long qn =
          base + stride + threadIdx.x < n ? base + stride + threadIdx.x : n - 1;
      rn = rho[qn];
      en = e[qn];
      if (tguess) gn = tguess[qn];
    }
    if (ML) {
      float x0, x1;
      mlp_inputs(ph, r, ee, x0, x1);
      g = mlp_guess_wave(ph, sMlp, x0, x1, lane);
    }
    double t = NAN;
    int iters = 0, fallback = 0;
    int rc = 1;
    if (r > 0.0 && ee > 0.0)
      rc = eos_temperature(ph, r, ee, g, ML ? ph.newton_maxit_mlp : ph.newton_maxit, t, iters,
                           fallback);
    if (!valid) continue;
    T[q] = t;
    if (T0) T0[q] = g;
    it += iters;
    mx = iters > mx ? iters : mx;
    fb += fallback;
    bad |= rc ? 2 : 0;
  }
  if (bad) atomicOr(flags, bad);
  if (!stats) return;  // block-uniform: no statistics requested
  // statistics: wave, then block totals, one set of atomics per block
  for (int o = 32; o > 0; o >>= 1) {
    it += __shfl_xor(it, o);
    fb += __shfl_xor(fb, o);
    const unsigned long long m2 = __shfl_xor(mx, o);
    mx = m2 > mx ? m2 : mx;
  }
  __shared__ unsigned long long s_st[3][4];
  const int wv = threadIdx.x >> 6;
  if (lane == 0) {
    s_st[0][wv] = it;
    s_st[1][wv] = mx;
    s_st[2][wv] = fb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, m = 0, f = 0;
    for (int w = 0; w < 4; ++w) {
      a += s_st[0][w];
      m = s_st[1][w] > m ? s_st[1][w] : m;
      f += s_st[2][w];
    }
    atomicAdd(&stats[0], a);
    atomicMax(&stats[1], m);
    atomicAdd(&stats[2], f);
  }
}

hipError_t launch_eos_solve(const Ctx &c, const double *rho, const double *e,
                            const double *tguess, long long n, double *T, double *T0,
                            bool stats) {
  long long nb = (n + 255) / 256;
  nb = nb < 8192 ? nb : 8192;
  unsigned long long *st = stats ? c.nstats : nullptr;
  if (c.d.eos_guess == MHD_GUESS_MLP)
    hipLaunchKernelGGL(eos_solve_kernel<true>, dim3((unsigned)nb), dim3(256), 0, c.stream, c.ph,
                       rho, e, tguess, n, c.mlp, T, T0, st, c.flags);
  else
    hipLaunchKernelGGL(eos_solve_kernel<false>, dim3((unsigned)nb), dim3(256), 0, c.stream, c.ph,
                       rho, e, tguess, n, c.mlp, T, T0, st, c.flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagnostics: div B (eq. divb), |B_face| max, conservation totals
// ---------------------------------------------------------------------------

constexpr int DIAG_BLOCKS = 1024;
constexpr int NDIAG = 9;  // divb max, divb^2 sum, |B| max, 5 totals, bflux_x0

__global__ __launch_bounds__(256) void diag_kernel(Phys ph, const double *__restrict__ U,
                                                   const double *__restrict__ Bx,
                                                   const double *__restrict__ By,
                                                   const double *__restrict__ Bz,
                                                   double *__restrict__ part) {
  const size_t plane = (size_t)ph.nx * ph.ny;
  const size_t n = plane * ph.nz;
  const double dmin = fmin(ph.dx, fmin(ph.dy, ph.dz));
  double v[NDIAG];
  for (int f = 0; f < NDIAG; ++f) v[f] = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(ph, q, i, j, k);
    const int ip = i + 1 == ph.nx ? 0 : i + 1;
    const int jp = j + 1 == ph.ny ? 0 : j + 1;
    const int kp = ph.reflect ? k + 1 : (k + 1 == ph.nz ? 0 : k + 1);
    const double bxl = Bx[q], bxr = Bx[q - i + ip];
    const double byl = By[q], byr = By[q + (size_t)(jp - j) * ph.nx];
    const double bzl = Bz[q], bzr = Bz[(size_t)kp * plane + (q - (size_t)k * plane)];
    const double d = ((bxr - bxl) * ph.idx + (byr - byl) * ph.idy + (bzr - bzl) * ph.idz) * dmin;
    v[0] = fmax(v[0], fabs(d));
    v[1] += d * d;
    v[2] = fmax(v[2], fmax(fabs(bxl), fmax(fabs(byl), fabs(bzl))));
    if (ph.reflect && k == ph.nz - 1) v[2] = fmax(v[2], fabs(bzr));
    for (int f = 0; f < 5; ++f) v[3 + f] += U[f * n + q];
    if (i == 0) v[8] += bxl;
  }
  __shared__ double sm[NDIAG][256];
  for (int f = 0; f < NDIAG; ++f) sm[f][threadIdx.x] = v[f];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sm[0][threadIdx.x] = fmax(sm[0][threadIdx.x], sm[0][threadIdx.x + s]);
      sm[2][threadIdx.x] = fmax(sm[2][threadIdx.x], sm[2][threadIdx.x + s]);
      sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
      for (int f = 3; f < NDIAG; ++f) sm[f][threadIdx.x] += sm[f][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < NDIAG) part[(size_t)threadIdx.x * DIAG_BLOCKS + blockIdx.x] = sm[threadIdx.x][0];
}

hipError_t launch_diagnostics(const Ctx &c, const double *U, const double *Bx,
                              const double *By, const double *Bz, double *out) {
  hipLaunchKernelGGL(diag_kernel, dim3(DIAG_BLOCKS), dim3(256), 0, c.stream, c.ph, U, Bx, By, Bz,
                     c.red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  static thread_local double host[NDIAG * DIAG_BLOCKS];
  e = hipMemcpyAsync(host, c.red, sizeof(double) * NDIAG * DIAG_BLOCKS, hipMemcpyDeviceToHost,
                     c.stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return e;
  // fixed-order host reduction of the block partials
  for (int f = 0; f < NDIAG; ++f) {
    long double s = 0.0L;
    double m = 0.0;
    for (int b = 0; b < DIAG_BLOCKS; ++b) {
      const double x = host[(size_t)f * DIAG_BLOCKS + b];
      if (f == 0 || f == 2)
        m = x > m ? x : m;
      else
        s += x;
    }
    out[f] = (f == 0 || f == 2) ? m : (double)s;
  }
  return hipSuccess;
}

__global__ void zero_walls_kernel(double *Bz, size_t plane, size_t top) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < plane;
       q += (size_t)gridDim.x * blockDim.x) {
    Bz[q] = 0.0;
    Bz[top + q] = 0.0;
  }
}

hipError_t launch_zero_walls(const Ctx &c, double *Bz) {
  const size_t plane = (size_t)c.ph.nx * c.ph.ny;
  int nb = (int)((plane + 255) / 256);
  nb = nb < 1024 ? nb : 1024;
  hipLaunchKernelGGL(zero_walls_kernel, dim3(nb), dim3(256), 0, c.stream, Bz, plane,
                     plane * (size_t)c.ph.nz);
  return hipGetLastError();
}

}  // namespace mhd
