// mhd_device.h -- device functions of the MHD stage: EOS, cons -> prim,
// reconstruction, the LHLLD flux in deviation form and the Contact-CT edge.
//
// Precision: R is the arithmetic type of reconstruction, Riemann flux and
// EMFs (double, or float in the split mode).  Cons -> prim, the EOS Newton
// solve and every accumulation run in double.
#pragma once

#include <hip/hip_runtime.h>

#include "mhd_internal.h"

namespace mhd {

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------

template <typename R> __device__ __forceinline__ R rcp(R x);
// FP64: hardware reciprocal refined by two Newton steps (about 1 ulp; the
// IEEE division sequence costs twice as many instructions)
template <> __device__ __forceinline__ double rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// split mode: hardware reciprocal (1 ulp), no IEEE division sequence
template <> __device__ __forceinline__ float rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <typename R> __device__ __forceinline__ R sqroot(R x);
// FP64: reciprocal square root refined by Goldschmidt/Newton steps; x >= 0
template <> __device__ __forceinline__ double sqroot<double>(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0;
}
template <> __device__ __forceinline__ float sqroot<float>(float x) {
  return __builtin_amdgcn_sqrtf(x);
}

// Reciprocal and square root of the flux arithmetic (slopes, wave speeds,
// star states).  FP64: one refinement step fewer than rcp / sqroot.  The
// hardware seeds are good to about 6e-8 relative; one Newton step brings
// the reciprocal to at most 11 ulp, one Goldschmidt step the square root to
// at most 36 ulp (measured on gfx950 over 2^20 arguments spread over
// 2^-200 .. 2^200), where the full sequences are correctly rounded or
// within half an ulp.  The flux quantities are differences of numbers many
// orders of magnitude coarser than that; exact zeros (a zero deviation, a
// zero slope) stay exact, since they come from the structure of the
// formulas, not from the precision of a reciprocal.  FP32: the hardware
// instructions, as rcp / sqroot.
template <typename R> __device__ __forceinline__ R rcp_flux(R x);
template <> __device__ __forceinline__ double rcp_flux<double>(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
template <> __device__ __forceinline__ float rcp_flux<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <typename R> __device__ __forceinline__ R sqroot_flux(R x);
template <> __device__ __forceinline__ double sqroot_flux<double>(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double g = x * y;
  const double r = fma(-g, 0.5 * y, 0.5);
  return x > 0.0 ? fma(g, r, g) : 0.0;
}
template <> __device__ __forceinline__ float sqroot_flux<float>(float x) {
  return __builtin_amdgcn_sqrtf(x);
}

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// The logical block of physical block bid: XCD j (bid = j, j+8, ...) takes
// the contiguous run [j q + min(j, r), ...) of the nblk logical blocks
// (q = nblk / 8, r = nblk mod 8), a bijection onto [0, nblk), so blocks that
// touch neighbouring data share one L2.
__device__ __forceinline__ int xcd_logical_block(int bid, int nblk) {
  const int q8 = nblk / 8, r8 = nblk % 8;
  const int xcd = bid % 8, slot = bid / 8;
  return xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
}

// Cells [c0, c1) of this block of a grid-wide per-cell kernel.  Blocks take
// contiguous chunks of whole blockDim-cell runs in XCD-contiguous logical
// order, so the rows and planes a cell's neighbours live in are read by
// blocks that share one L2.
__device__ __forceinline__ void block_cells(size_t n, size_t &c0, size_t &c1) {
  const size_t span = (size_t)gridDim.x * blockDim.x;
  const size_t per = (n + span - 1) / span * blockDim.x;
  c0 = (size_t)xcd_logical_block(blockIdx.x, gridDim.x) * per;
  c1 = c0 + per < n ? c0 + per : n;
}

// (i, j, k) of a linear cell index q < nx ny nz (< 2^32: three state
// copies of a larger grid would not fit in HBM), with 32-bit divisions
__device__ __forceinline__ void cell_ijk(const Phys &ph, size_t q, int &i, int &j, int &k) {
  const unsigned u = (unsigned)q, nx = (unsigned)ph.nx, ny = (unsigned)ph.ny;
  const unsigned r = u / nx;
  i = (int)(u - r * nx);
  k = (int)(r / ny);
  j = (int)(r - (unsigned)k * ny);
}

// ---------------------------------------------------------------------------
// gas + radiation EOS (Sect. 2.2, eqs. prad, erad)
// e_int(T) = C_g T + (a/rho) T^4, P = rho (R/mu) T + a T^4 / 3
// ---------------------------------------------------------------------------

// Newton T <- T + de / c_v from the guess, stopping when |de| < tol e before
// an update; a non-finite / non-positive guess or the iteration cap falls
// back to a safeguarded Newton-bisection on the closed-form bracket
// [min(e/(2C_g), (rho e/(2a))^1/4), min(e/C_g, (rho e/a)^1/4)].
// Returns 0, or 2 when even the bracketed solve did not converge.
__device__ __forceinline__ int eos_temperature(const Phys &ph, double rho,
                                               double e, double tguess, int maxit,
                                               double &T, int &iters,
                                               int &fallback) {
  // the Newton step divides by c_v > 0 with the refined reciprocal (a few
  // ulp); the stopping test on |de| decides the result's accuracy
  const double cg = ph.cg, ar = ph.arad * rcp<double>(rho), tol = ph.newton_tol * e;
  iters = 0;
  fallback = 0;
  double t = tguess;
  if (t > 0.0 && t < INFINITY) {
    for (int n = 0; n < maxit; ++n) {
      const double t3 = t * t * t;
      const double de = e - (cg * t + ar * t3 * t);
      if (fabs(de) < tol) {
        T = t;
        iters = n;
        return 0;
      }
      t = t + de * rcp<double>(cg + 4.0 * ar * t3);
      iters = n + 1;
      if (!(t > 0.0 && t < INFINITY)) break;
    }
  }
  fallback = 1;
  const double ecg = e * ph.icg, ear = e * rcp<double>(ar);
  double lo = fmin(0.5 * ecg, sqroot<double>(sqroot<double>(0.5 * ear)));
  double hi = fmin(ecg, sqroot<double>(sqroot<double>(ear)));
  t = 0.5 * (lo + hi);
  for (int n = 0; n < 400; ++n) {
    const double t3 = t * t * t;
    const double de = e - (cg * t + ar * t3 * t);
    if (fabs(de) < tol) {
      T = t;
      return 0;
    }
    if (de > 0.0)
      lo = t;
    else
      hi = t;
    const double tn = t + de * rcp<double>(cg + 4.0 * ar * t3);
    t = (tn > lo && tn < hi) ? tn : 0.5 * (lo + hi);
    if (hi - lo <= 8.881784197001252e-16 * hi) {
      T = t;
      return 0;
    }
  }
  T = t;
  return 2;
}

// P, and the auxiliary indices gamma_e = P/(rho e) + 1, gamma_c = rho c_s^2/P
// with c_s^2 = (dP/drho)_T + T (dP/dT)_rho^2 / (rho^2 c_v).
__device__ __forceinline__ void eos_thermo(const Phys &ph, double rho, double ir, double e,
                                           double T, double &P, double &ge,
                                           double &gc) {
  const double t3 = T * T * T;
  P = rho * ph.rmu * T + ph.arad * t3 * T * (1.0 / 3.0);
  const double cv = ph.cg + 4.0 * ph.arad * t3 * ir;
  const double dpdt = rho * ph.rmu + (4.0 / 3.0) * ph.arad * t3;
  const double cs2 = ph.rmu * T + T * dpdt * dpdt * (ir * ir) * rcp<double>(cv);
  ge = P * ir * rcp<double>(e) + 1.0;
  gc = rho * cs2 * rcp<double>(P);
}

// ---------------------------------------------------------------------------
// cons -> prim of one cell (double); deviation from the background
// ---------------------------------------------------------------------------

// Cell fields in the order used everywhere below.
enum { Q_RHO = 0, Q_VX, Q_VY, Q_VZ, Q_P, Q_BX, Q_BY, Q_BZ, Q_GE, Q_GC };

struct PrimOut {
  double w[10];  // deviations of rho, P, gamma_e, gamma_c; full v, B_cc
  double T;
  int iters, fallback;
  int bad;       // 1 unphysical, 2 EOS failure
};

// forward EOS: e_int(rho, T) = C_g T + a T^4 / rho (eq. erad)
__device__ __forceinline__ double specific_eint_rt(const Phys &ph, double rho, double T) {
  return ph.cg * T + ph.arad * T * T * T * T * rcp<double>(rho);
}

// specific internal energy e_int = (E - rho v^2/2 - B_cc^2/2) / rho
__device__ __forceinline__ double specific_eint(const double u[5], const double b[3]) {
  const double rho = u[0];
  const double ir = rcp<double>(rho);
  const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
  const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  return (u[4] - 0.5 * rho * (vx * vx + vy * vy + vz * vz) - 0.5 * b2) * ir;
}

// u: conserved (rho, m, E); b: cell-centred field; bg: background
// (rho, P, gamma_e, gamma_c) of the cell's height.
template <bool GR>
__device__ __forceinline__ void cons2prim(const Phys &ph, const double u[5],
                                          const double b[3], double tguess,
                                          const double bg[4], PrimOut &o,
                                          int maxit = -1) {
  const double rho = u[0];
  const double ir = rcp<double>(rho);
  const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
  const double e = specific_eint(u, b);
  o.bad = (rho > 0.0 && e > 0.0 && e < INFINITY) ? 0 : 1;
  double P, ge = ph.gamma, gc = ph.gamma;
  o.T = 0.0;
  o.iters = 0;
  o.fallback = 0;
  if (GR) {
    double T = tguess;
    if (!o.bad) {
      if (eos_temperature(ph, rho, e, tguess, maxit < 0 ? ph.newton_maxit : maxit, T, o.iters,
                          o.fallback))
        o.bad = 2;
    }
    o.T = T;
    eos_thermo(ph, rho, ir, e, T, P, ge, gc);
  } else {
    P = ph.gm1 * rho * e;
  }
  o.w[Q_RHO] = rho - bg[0];
  o.w[Q_VX] = vx;
  o.w[Q_VY] = vy;
  o.w[Q_VZ] = vz;
  o.w[Q_P] = P - bg[1];
  o.w[Q_BX] = b[0];
  o.w[Q_BY] = b[1];
  o.w[Q_BZ] = b[2];
  o.w[Q_GE] = ge - bg[2];
  o.w[Q_GC] = gc - bg[3];
}

// ---------------------------------------------------------------------------
// learned initial guess of T(rho, e_int) on the matrix cores
//
// A 2 -> 64 -> 64 -> 1 ReLU network evaluated for 32 cells per pass.
// Layer 1 runs on v_mfma_f32_32x32x8_bf16 (A 32x8, B 8x32, D 32x32, FP32
// accumulation), layer 2 on gfx950's v_mfma_f32_32x32x16_bf16 (K = 16 per
// instruction at the same instruction time: half the passes).  Operand
// layout of the K = 8 form (lane l, t = 0..3, r = 0..15):
//   A: A[l%32][4(l/32) + t]     B: B[4(l/32) + t][l%32]
//   D: row 8(r/4) + 4(l/32) + r%4, column l%32
// so the accumulator of one layer, taken four registers at a time, holds
// the hidden units 8j + 4(l/32) + 0..3 of its column (rows = hidden units,
// columns = cells).  The K = 16 form takes eight values per lane and each
// lane half supplies its own eight K rows, the same way in A and in B; so
// the B operand of K block q is the two four-register groups 2q and 2q+1 of
// the layer-1 accumulator as they are, and the A operand (W2) is packed with
// the matching hidden units: value t of lane l is unit
// 8(2q + t/4) + 4(l/32) + t%4.  Layer 1 folds its bias into K = 8 rows
// (x0h, x0h, x0l, x1h | x1h, x1l, 1, 1) against (w0h, w0l, w0h, w1h | w1l,
// w1h, b1h, b1l): hi/lo BF16 pairs keep about 16 bits of the inputs and of
// W1, b1.  Layer 3 (64 -> 1) takes BF16 dot products of the layer-2
// registers with W3 pairs on the vector unit.
// ---------------------------------------------------------------------------

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

struct MlpLds {        // host-packed fragments, staged in LDS per block
  v4s a1[2][64];       // layer 1, per output block mb and lane
  v8s a2[2][4][64];    // layer 2: W2[32mb + l%32][8(2q + t/4) + 4(l/32) + t%4]
  float c2[2][16][64]; // layer-2 accumulator start: b2 in the D layout
  short w3[64];        // layer 3 weights (BF16 bits)
};

typedef short v2s __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }
// two FP32 values to one register of packed BF16 (round to nearest even),
// a in the low half: one v_cvt_pk_bf16_f32
__device__ __forceinline__ unsigned pack2_bf16(float a, float b) {
  v2bf r;
  r[0] = (__bf16)a;
  r[1] = (__bf16)b;
  return __builtin_bit_cast(unsigned, r);
}
__device__ __forceinline__ v4s pack_bf16(float a, float b, float c, float d) {
  const v2u w = {pack2_bf16(a, b), pack2_bf16(c, d)};
  return __builtin_bit_cast(v4s, w);
}

// ReLU of two FP32 values into one register of packed BF16: the pair is
// converted in one instruction, then a negative BF16 (a negative 16-bit
// integer, -0 included) is cleared by an integer max with 0 on both halves
// (v_pk_max_i16).  The empty asm statement (no instruction) hides the
// packed register from the instruction combiner, which would otherwise
// split the pair into two single conversions and a permute.
__device__ __forceinline__ unsigned pack2_relu(float a, float b) {
  unsigned u = pack2_bf16(a, b);
  asm("" : "+v"(u));
  return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(v2s, u), (v2s)0));
}
__device__ __forceinline__ v4s pack_relu(const v16f &d, int j) {
  const v2u w = {pack2_relu(d[4 * j], d[4 * j + 1]), pack2_relu(d[4 * j + 2], d[4 * j + 3])};
  return __builtin_bit_cast(v4s, w);
}

// One pass over the 32 cells held by lanes 0..31 (lanes l and l+32 carry
// the inputs of cell l%32).  Returns the network output (without b3) of
// cell l%32 on every lane.  Must be called by all 64 lanes.
__device__ __forceinline__ float mlp_pass(const MlpLds &S, float x0, float x1, int lane) {
  const float x0h = bf16_round(x0), x1h = bf16_round(x1);
  const v4s b = lane < 32 ? pack_bf16(x0h, x0h, x0 - x0h, x1h)
                          : pack_bf16(x1h, x1 - x1h, 1.0f, 1.0f);
  const v16f z = {};
  const v16f c0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(S.a1[0][lane], b, z, 0, 0, 0);
  const v16f c1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(S.a1[1][lane], b, z, 0, 0, 0);
  v4s h[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    h[j] = pack_relu(c0, j);
    h[4 + j] = pack_relu(c1, j);
  }
  v16f d0, d1;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    d0[r] = S.c2[0][r][lane];
    d1[r] = S.c2[1][r][lane];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const v8s hq = __builtin_shufflevector(h[2 * q], h[2 * q + 1], 0, 1, 2, 3, 4, 5, 6, 7);
    const v8bf b = __builtin_bit_cast(v8bf, hq);
    d0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, S.a2[0][q][lane]), b,
                                                 d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, S.a2[1][q][lane]), b,
                                                 d1, 0, 0, 0);
  }
  // layer 3, 64 -> 1: this lane holds hidden units 8j + 4(l/32) + t (d0)
  // and 32 + the same (d1) of its cell; BF16 dot products of register pairs
  // with the matching W3 pairs, then the other half of the wave's rows
  const int kh = 4 * (lane >> 5);
  float y = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const v4s hj = j < 4 ? pack_relu(d0, j) : pack_relu(d1, j - 4);
    const int row = (j < 4 ? 8 * j : 32 + 8 * (j - 4)) + kh;
    const v2s wlo = *reinterpret_cast<const v2s *>(&S.w3[row]);
    const v2s whi = *reinterpret_cast<const v2s *>(&S.w3[row + 2]);
    const v2s hlo = {hj[0], hj[1]}, hhi = {hj[2], hj[3]};
    y = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2bf, hlo),
                                        __builtin_bit_cast(v2bf, wlo), y, false);
    y = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2bf, hhi),
                                        __builtin_bit_cast(v2bf, whi), y, false);
  }
  return y + __shfl_xor(y, 32);
}

// Network inputs of one cell: normalised log10 rho and log10 e, clipped to
// the training box [-1, 1].
__device__ __forceinline__ void mlp_inputs(const Phys &ph, double rho, double e, float &x0,
                                           float &x1) {
  const float l2 = 0.30102999566398120f;  // log10(2)
  x0 = (__log2f((float)rho) * l2 - ph.mlp_norm[0]) * ph.mlp_norm[1];
  x1 = (__log2f((float)e) * l2 - ph.mlp_norm[2]) * ph.mlp_norm[3];
  x0 = fminf(fmaxf(x0, -1.0f), 1.0f);
  x1 = fminf(fmaxf(x1, -1.0f), 1.0f);
  if (!(x0 == x0)) x0 = 0.0f;  // NaN inputs of non-physical cells
  if (!(x1 == x1)) x1 = 0.0f;
}

// Temperature guess from the network output y: log10 T = (y + b3)/s_T + c_T.
__device__ __forceinline__ double mlp_temperature(const Phys &ph, float y) {
  const float lg = (y + ph.mlp_b3) * ph.mlp_inv_sT + ph.mlp_norm[4];
  return (double)exp2f(lg * 3.32192809488736235f);
}

// Guess for the cells held by all 64 lanes of the wave (two passes).
__device__ __forceinline__ double mlp_guess_wave(const Phys &ph, const MlpLds &S, float x0,
                                                 float x1, int lane) {
  const float o0 = __shfl_xor(x0, 32), o1 = __shfl_xor(x1, 32);
  const bool lo = lane < 32;
  const float y0 = mlp_pass(S, lo ? x0 : o0, lo ? x1 : o1, lane);  // cells 0..31
  const float y1 = mlp_pass(S, lo ? o0 : x0, lo ? o1 : x1, lane);  // cells 32..63
  return mlp_temperature(ph, lo ? y0 : y1);
}


// ---------------------------------------------------------------------------
// reconstruction (Sect. 2.5): van Leer slope, harmonic form
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R vanleer(R a, R b) {
  const R ab = a * b;
  if constexpr (sizeof(R) == 4) {
    // branch-free (a + b is nonzero whenever ab > 0, the only case used)
    const R q = R(2) * ab * rcp_flux<R>(a + b);
    return ab > R(0) ? q : R(0);
  } else {
    // FP64: the reciprocal sequence only where a lane needs it (keeps the
    // register pressure of the unrolled reconstruction down)
    return ab > R(0) ? R(2) * ab * rcp_flux<R>(a + b) : R(0);
  }
}

// ---------------------------------------------------------------------------
// LHLLD flux in deviation form (Sect. 2.6 and 2.8)
//
// One side of the face in the face frame (normal n, transverse t1, t2):
// deviations of rho, P, gamma_e, gamma_c from the face background and the
// full velocity and transverse field (the background has none).  The result
// is F(W_L, W_R) - F(W_hat_f, W_hat_f) in the order {mass, mom_n, mom_t1,
// mom_t2, energy, B_t1, B_t2}: with p~ = p_T - P_hat the background pressure
// enters only through E + P_hat, so a zero deviation gives exactly zero.
// ---------------------------------------------------------------------------

template <typename R>
struct Side {
  R drho, vn, v1, v2, dp, b1, b2, dge, dgc;
};

template <typename R>
struct FaceBg {
  R rho, p, ge, gc;
};

template <typename R>
struct SideQ {  // derived side quantities
  R rho, vn, v1, v2, pt, b1, b2;
};

// Reciprocals of two numbers.  FP64: one hardware reciprocal with its
// Newton steps serves both (1/a = b/(ab)); FP32: the hardware reciprocal is
// a single instruction, so each is taken directly.
template <typename R>
__device__ __forceinline__ void rcp2(R a, R b, R &ia, R &ib) {
  if constexpr (sizeof(R) == 8) {
    const R r = rcp_flux<R>(a * b);
    ia = b * r;
    ib = a * r;
  } else {
    ia = rcp_flux<R>(a);
    ib = rcp_flux<R>(b);
  }
}

// Side quantities from the reconstructed deviations; ir = 1/rho comes from
// the caller (taken for both sides at once).  Returns the fast speed along
// the normal, c_s^2 and |v|^2.
template <typename R, bool GR>
__device__ __forceinline__ void side_prep(const Side<R> &s, R bn, const FaceBg<R> &bg, R rho,
                                          R ir, R gam, SideQ<R> &q, R &cf, R &cs2, R &v2) {
  q.rho = rho;
  q.vn = s.vn;
  q.v1 = s.v1;
  q.v2 = s.v2;
  q.b1 = s.b1;
  q.b2 = s.b2;
  const R P = bg.p + s.dp;
  const R bn2 = bn * bn;
  const R B2 = bn2 + s.b1 * s.b1 + s.b2 * s.b2;
  v2 = s.vn * s.vn + s.v1 * s.v1 + s.v2 * s.v2;
  const R gc = GR ? bg.gc + s.dgc : gam;
  q.pt = s.dp + R(0.5) * B2;  // p_T - P_hat
  cs2 = gc * P * ir;
  const R a2b2 = cs2 + B2 * ir;
  // discriminant clipped at zero against rounding (fmax: also maps NaN to 0)
  const R disc = fmax(a2b2 * a2b2 - R(4) * cs2 * bn2 * ir, R(0));
  cf = sqroot_flux<R>(R(0.5) * (a2b2 + sqroot_flux<R>(disc)));
}

// Total energy, v.B and the physical flux (deviation form) of one side;
// igm = 1/(gamma_e - 1), v2 = |v|^2 and pt = p_T - P_hat as from side_prep.
// The LHLLD solver needs them for the side it selects only.
template <typename R>
__device__ __forceinline__ void side_flux(const Side<R> &s, R bn, const FaceBg<R> &bg, R rho,
                                          R igm, R v2, R pt, R &E, R &vb, R F[7]) {
  const R P = bg.p + s.dp;
  const R bn2 = bn * bn;
  const R B2 = bn2 + s.b1 * s.b1 + s.b2 * s.b2;
  E = P * igm + R(0.5) * rho * v2 + R(0.5) * B2;
  vb = s.vn * bn + s.v1 * s.b1 + s.v2 * s.b2;
  const R rv = rho * s.vn;
  F[0] = rv;
  F[1] = rv * s.vn + pt - bn2;
  F[2] = rv * s.v1 - bn * s.b1;
  F[3] = rv * s.v2 - bn * s.b2;
  F[4] = (E + bg.p + pt) * s.vn - bn * vb;
  F[5] = s.vn * s.b1 - bn * s.v1;
  F[6] = s.vn * s.b2 - bn * s.v2;
}

template <typename R>
struct Star {  // single-star state of one side, as differences from U
  R rho, drho;     // rho*, rho* - rho
  R dv1, dv2;      // v*_t - v_t
  R db1, db2;      // B*_t - B_t
  R isd, dvn;      // 1/(S - S_M), S_M - v_n
};

// Density, transverse velocity and field of the single-star state of one
// side (Miyoshi & Kusano 2005), every difference U* - U written so that no
// large number is subtracted from another (the split mode depends on it).
// isd = 1/(S - S_M) comes from the caller; iD = 1/D of a non-degenerate side.
template <typename R>
__device__ __forceinline__ void star_side(const SideQ<R> &q, R S, R SM, R bn, R isd, R svn,
                                          bool nondeg, R iD, Star<R> &st) {
  const R f = q.rho * isd;
  const R dvn = SM - q.vn;
  st.isd = isd;
  st.dvn = dvn;
  st.rho = f * svn;
  st.drho = f * dvn;
  // degenerate (|D| <= 1e-8 rho (S - v_n)^2): v_t and B_t unchanged
  const R qv = nondeg ? bn * dvn * iD : R(0);           // v*_t - v_t = -B_t qv
  const R qb = nondeg ? q.rho * svn * dvn * iD : R(0);  // B*_t - B_t = B_t qb
  st.dv1 = -q.b1 * qv;
  st.dv2 = -q.b2 * qv;
  st.db1 = q.b1 * qb;
  st.db2 = q.b2 * qb;
}

template <typename R>
__device__ __forceinline__ R sel(bool c, R a, R b) { return c ? a : b; }

// LHLLD flux in deviation form.  The fan is resolved without branches: the
// side of the contact that holds x/t = 0 (S_M >= 0: left) is selected, and
// its single- and double-star fluxes are built once.
template <typename R, bool GR>
__device__ __forceinline__ void riemann(const Side<R> &L, const Side<R> &Rt,
                                        R bn, const FaceBg<R> &bg, R gam,
                                        R igm1, int xi_mode, R mcut, R imcut,
                                        R F[7]) {
  const R rhoL = bg.rho + L.drho, rhoR = bg.rho + Rt.drho;
  R irL, irR, igL = igm1, igR = igm1;
  rcp2<R>(rhoL, rhoR, irL, irR);
  if (GR) rcp2<R>(bg.ge + L.dge - R(1), bg.ge + Rt.dge - R(1), igL, igR);
  SideQ<R> qL, qR;
  R cfL, cfR, csL, csR, v2L, v2R;
  side_prep<R, GR>(L, bn, bg, rhoL, irL, gam, qL, cfL, csL, v2L);
  side_prep<R, GR>(Rt, bn, bg, rhoR, irR, gam, qR, cfR, csR, v2R);
  const R cmax = fmax(cfL, cfR);
  const R SL = fmin(qL.vn, qR.vn) - cmax;
  const R SR = fmax(qL.vn, qR.vn) + cmax;
  const R svnL = SL - qL.vn, svnR = SR - qR.vn;
  const R aL = svnL * qL.rho, aR = svnR * qR.rho;
  const R iden = rcp_flux<R>(aR - aL);
  const R SM = (aR * qR.vn - aL * qL.vn - qR.pt + qL.pt) * iden;
  // low-dissipation factor xi on the upwind term of p_T* (sonic Mach)
  R xi = R(1);
  if (xi_mode != MHD_XI_OFF) {
    R m2;
    if constexpr (sizeof(R) == 8) {
      // max(v_L^2/c_L^2, v_R^2/c_R^2) with one reciprocal
      m2 = fmax(v2L * csR, v2R * csL) * rcp_flux<R>(csL * csR);
    } else {
      m2 = fmax(v2L * rcp_flux<R>(csL), v2R * rcp_flux<R>(csR));
    }
    const R M = sqroot_flux<R>(m2);
    if (xi_mode == MHD_XI_LINEAR)
      xi = fmin(M * imcut, R(1));
    else
      xi = M < mcut ? M : R(1);
  }
  const R pst = (aR * qL.pt - aL * qR.pt + xi * qL.rho * qR.rho * svnR * svnL * (qR.vn - qL.vn)) *
                iden;
  // single-star states of both sides
  R isdL, isdR;
  rcp2<R>(SL - SM, SR - SM, isdL, isdR);
  const R bn2 = bn * bn;
  const R DL = qL.rho * svnL * (SL - SM) - bn2, DR = qR.rho * svnR * (SR - SM) - bn2;
  const bool ndL = fabs(DL) > R(1e-8) * qL.rho * svnL * svnL;
  const bool ndR = fabs(DR) > R(1e-8) * qR.rho * svnR * svnR;
  R iDL, iDR;
  rcp2<R>(ndL ? DL : R(1), ndR ? DR : R(1), iDL, iDR);
  Star<R> sL, sR;
  star_side<R>(qL, SL, SM, bn, isdL, svnL, ndL, iDL, sL);
  star_side<R>(qR, SR, SM, bn, isdR, svnR, ndR, iDR, sR);
  // Alfven waves: sqrt(rho*) of both sides, 1/sqrt(rho*) and 1/(sum)
  const R sqL = sqroot_flux<R>(sL.rho), sqR = sqroot_flux<R>(sR.rho);
  R isqL, isqR, is;
  if constexpr (sizeof(R) == 8) {
    const R pr = sqL * sqR, sm = sqL + sqR;
    const R r = rcp_flux<R>(pr * sm);
    isqL = sqR * sm * r;
    isqR = sqL * sm * r;
    is = pr * r;
  } else {
    isqL = rcp_flux<R>(sqL);
    isqR = rcp_flux<R>(sqR);
    is = rcp_flux<R>(sqL + sqR);
  }
  const R abn = fabs(bn);
  const R SsL = SM - abn * isqL;
  const R SsR = SM + abn * isqR;
  // double-star transverse velocity and field
  const R sg = bn >= R(0) ? R(1) : R(-1);
  const R vL1 = qL.v1 + sL.dv1, vL2 = qL.v2 + sL.dv2, vR1 = qR.v1 + sR.dv1, vR2 = qR.v2 + sR.dv2;
  const R bL1 = qL.b1 + sL.db1, bL2 = qL.b2 + sL.db2, bR1 = qR.b1 + sR.db1, bR2 = qR.b2 + sR.db2;
  const R w1 = (sqL * vL1 + sqR * vR1 + (bR1 - bL1) * sg) * is;
  const R w2 = (sqL * vL2 + sqR * vR2 + (bR2 - bL2) * sg) * is;
  const R c1 = (sqL * bR1 + sqR * bL1 + sqL * sqR * (vR1 - vL1) * sg) * is;
  const R c2 = (sqL * bR2 + sqR * bL2 + sqL * sqR * (vR2 - vL2) * sg) * is;
  const R vbss = SM * bn + w1 * c1 + w2 * c2;
  // region (eq. flux-hlld): outside the fan, or inside on the side of the
  // contact that holds x/t = 0, single or double star
  const bool outL = R(0) <= SL, outR = SR < R(0);
  const bool lf = outL || (!outR && SM >= R(0));
  const bool fan = !(outL || outR);
  const bool dstar = lf ? (SsL < R(0)) : (R(0) <= SsR);
  const R S = sel(lf, SL, SR), Ss = sel(lf, SsL, SsR), sq = sel(lf, sqL, sqR);
  const R rho = sel(lf, qL.rho, qR.rho);
  const R rs = sel(lf, sL.rho, sR.rho), drs = sel(lf, sL.drho, sR.drho);
  const R dv1 = sel(lf, sL.dv1, sR.dv1), dv2 = sel(lf, sL.dv2, sR.dv2);
  const R db1 = sel(lf, sL.db1, sR.db1), db2 = sel(lf, sL.db2, sR.db2);
  const R vs1 = sel(lf, vL1, vR1), vs2 = sel(lf, vL2, vR2);
  const R bs1 = sel(lf, bL1, bR1), bs2 = sel(lf, bL2, bR2);
  // energy, v.B and flux of the selected side
  const R pt = sel(lf, qL.pt, qR.pt), vn = sel(lf, qL.vn, qR.vn);
  Side<R> sa;
  sa.vn = vn;
  sa.v1 = sel(lf, qL.v1, qR.v1);
  sa.v2 = sel(lf, qL.v2, qR.v2);
  sa.b1 = sel(lf, qL.b1, qR.b1);
  sa.b2 = sel(lf, qL.b2, qR.b2);
  sa.dp = sel(lf, L.dp, Rt.dp);
  R E, vb, Fa[7];
  side_flux<R>(sa, bn, bg, rho, sel(lf, igL, igR), sel(lf, v2L, v2R), pt, E, vb, Fa);
  // E* - E of the selected side:
  // [(S_M - v_n)(E + P_hat) + p~* S_M - p~ v_n + B_n (v.B - v*.B*)] / (S - S_M)
  const R isd = sel(lf, sL.isd, sR.isd);
  const R dvn = sel(lf, sL.dvn, sR.dvn);
  const R vbs = SM * bn + vs1 * bs1 + vs2 * bs2;
  const R dE = (dvn * (E + bg.p) + pst * SM - pt * vn + bn * (vb - vbs)) * isd;
  // single-star flux F* = F + S (U* - U); the interface pressure p~*
  // carries the low-dissipation factor into the normal momentum;
  // double-star flux F** = F* + S* (U** - U*)
  const R esg = lf ? -sg : sg;
  R Fs[7], Fss[7];
  Fs[0] = Fa[0] + S * drs;
  Fs[1] = rs * SM * SM + pst - bn2;
  Fs[2] = Fa[2] + S * (drs * vs1 + rho * dv1);
  Fs[3] = Fa[3] + S * (drs * vs2 + rho * dv2);
  Fs[4] = Fa[4] + S * dE;
  Fs[5] = Fa[5] + S * db1;
  Fs[6] = Fa[6] + S * db2;
  Fss[2] = Fs[2] + Ss * rs * (w1 - vs1);
  Fss[3] = Fs[3] + Ss * rs * (w2 - vs2);
  Fss[4] = Fs[4] + Ss * sq * (vbs - vbss) * esg;
  Fss[5] = Fs[5] + Ss * (c1 - bs1);
  Fss[6] = Fs[6] + Ss * (c2 - bs2);
  F[0] = fan ? Fs[0] : Fa[0];
  F[1] = fan ? Fs[1] : Fa[1];
#pragma unroll
  for (int c = 2; c < 7; ++c) F[c] = fan ? (dstar ? Fss[c] : Fs[c]) : Fa[c];
}

// HLL flux (Harten, Lax & van Leer 1983) in the same deviation form, the
// solver of faces next to a flattened cell (Sect. 2.7): one state between
// the fastest waves, with the wave speeds of the LHLLD solver.  U_R - U_L
// is formed from the deviations, so that no background value is subtracted
// from another: the thermal energy difference is
// P_hat (g_L - g_R) i_L i_R + dP_R i_R - dP_L i_L (i = 1/(gamma_e - 1),
// g = gamma_e deviation) with the gas+radiation EOS, (dP_R - dP_L) i else.
template <typename R, bool GR>
__device__ __forceinline__ void hll_flux(const Side<R> &L, const Side<R> &Rt, R bn,
                                         const FaceBg<R> &bg, R gam, R igm1, R F[7]) {
  const R rhoL = bg.rho + L.drho, rhoR = bg.rho + Rt.drho;
  R irL, irR, igL = igm1, igR = igm1;
  rcp2<R>(rhoL, rhoR, irL, irR);
  if (GR) rcp2<R>(bg.ge + L.dge - R(1), bg.ge + Rt.dge - R(1), igL, igR);
  SideQ<R> qL, qR;
  R cfL, cfR, csL, csR, v2L, v2R;
  side_prep<R, GR>(L, bn, bg, rhoL, irL, gam, qL, cfL, csL, v2L);
  side_prep<R, GR>(Rt, bn, bg, rhoR, irR, gam, qR, cfR, csR, v2R);
  R EL, ER, vbL, vbR, FL[7], FR[7];
  side_flux<R>(L, bn, bg, rhoL, igL, v2L, qL.pt, EL, vbL, FL);
  side_flux<R>(Rt, bn, bg, rhoR, igR, v2R, qR.pt, ER, vbR, FR);
  const R cmax = fmax(cfL, cfR);
  const R SL = fmin(qL.vn, qR.vn) - cmax;
  const R SR = fmax(qL.vn, qR.vn) + cmax;
  const R eth = GR ? bg.p * (L.dge - Rt.dge) * igL * igR + Rt.dp * igR - L.dp * igL
                   : (Rt.dp - L.dp) * igm1;
  R dU[7];
  dU[0] = Rt.drho - L.drho;
  dU[1] = rhoR * Rt.vn - rhoL * L.vn;
  dU[2] = rhoR * Rt.v1 - rhoL * L.v1;
  dU[3] = rhoR * Rt.v2 - rhoL * L.v2;
  dU[4] = eth + R(0.5) * (rhoR * v2R - rhoL * v2L) +
          R(0.5) * ((Rt.b1 * Rt.b1 + Rt.b2 * Rt.b2) - (L.b1 * L.b1 + L.b2 * L.b2));
  dU[5] = Rt.b1 - L.b1;
  dU[6] = Rt.b2 - L.b2;
  const R iw = rcp_flux<R>(SR - SL);
  const bool outL = R(0) <= SL, outR = SR < R(0);
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    const R fh = (SR * FL[c] - SL * FR[c] + SL * SR * dU[c]) * iw;
    F[c] = outL ? FL[c] : (outR ? FR[c] : fh);
  }
}

// Face flux: HLL where the face touches a flattened cell, LHLLD elsewhere.
// The two solvers run under a lane mask, so their registers are not live
// at the same time.
template <typename R, bool GR>
__device__ __forceinline__ void face_flux(bool hll, const Side<R> &L, const Side<R> &Rt, R bn,
                                          const FaceBg<R> &bg, R gam, R igm1, int xi_mode,
                                          R mcut, R imcut, R F[7]) {
  if (hll)
    hll_flux<R, GR>(L, Rt, bn, bg, gam, igm1, F);
  else
    riemann<R, GR>(L, Rt, bn, bg, gam, igm1, xi_mode, mcut, imcut, F);
}

// ---------------------------------------------------------------------------
// Contact-CT edge EMF (Sect. 2.4; Gardiner & Stone 2005).
// Edge of component c with a = c+1, b = c+2 (cyclic) at (a-1/2, b-1/2):
//   Ea_b, Ea_bm : EMF on the a-faces at b and b-1
//   Eb_a, Eb_am : EMF on the b-faces at a and a-1
//   r_xy        : cell reference EMF -(v x B) at (a or a-1, b or b-1)
//   m_*         : mass flux through the matching face (upwind direction)
// Each face value is carried to the edge with the cell-side gradient of the
// upwind cell; the mean of the four is the edge EMF.
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R upwind(R m, R up, R dn) {
  const R mid = R(0.5) * (up + dn);  // branch-free selection
  const R side = m > R(0) ? up : dn;
  return m == R(0) ? mid : side;
}

template <typename R>
__device__ __forceinline__ R ct_edge(R Ea_b, R Ea_bm, R Eb_a, R Eb_am, R r_ab,
                                     R r_amb, R r_abm, R r_ambm, R m_ab,
                                     R m_abm, R m_ba, R m_bam) {
  const R d1 = upwind<R>(m_ab, Eb_am - r_amb, Eb_a - r_ab);
  const R d2 = upwind<R>(m_abm, Eb_am - r_ambm, Eb_a - r_abm);
  const R d3 = upwind<R>(m_ba, Ea_bm - r_abm, Ea_b - r_ab);
  const R d4 = upwind<R>(m_bam, Ea_bm - r_ambm, Ea_b - r_amb);
  return R(0.25) * ((Ea_b + Ea_bm) + (Eb_a + Eb_am)) + R(0.25) * ((d1 + d2) + (d3 + d4));
}

}  // namespace mhd
