// Device-side helpers shared by the pair and adjoint kernels (internal).
#pragma once

#include "md_internal.h"

namespace mdcell {

// ---------------------------------------------------------------- arithmetic helpers
// Reciprocal and reciprocal square root: the hardware estimate refined by Newton-Raphson
// iterations (r <- r + r (1 - x r); y <- y + y (1 - x y^2) / 2), once in FP32, twice / three
// times in FP64.
template <typename R> __device__ __forceinline__ R rcp_nr(R x);
template <> __device__ __forceinline__ float rcp_nr<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  const float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}
template <> __device__ __forceinline__ double rcp_nr<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <typename R> __device__ __forceinline__ R rsq_nr(R x);
template <> __device__ __forceinline__ float rsq_nr<float>(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  const float h = x * y;
  const float e = fmaf(-h, y, 1.0f);
  return fmaf(0.5f * y, e, y);
}
template <> __device__ __forceinline__ double rsq_nr<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

template <typename R> __device__ __forceinline__ void addto(double &a, R x) { a += (double)x; }

// LJ force scalar fs = 24 eps s^6 (2 s^6 - 1) / r^2 (force on i = fs * r_ij), evaluated in R from
// the FP64 squared distance.  FP32: one hardware reciprocal (1 ulp), no refinement -- the force
// error budget is 1e-5 relative.  FP64: reciprocal refined by two Newton steps.
template <typename R> __device__ __forceinline__ double lj_force_scalar(double r2, R eps24, R sig2);
template <> __device__ __forceinline__ double lj_force_scalar<float>(double r2, float eps24, float sig2) {
  const float ir2 = __builtin_amdgcn_rcpf((float)r2);
  const float s2 = sig2 * ir2;
  const float s6 = s2 * s2 * s2;
  return (double)((eps24 * ir2) * (s6 * fmaf(2.0f, s6, -1.0f)));
}
template <> __device__ __forceinline__ double lj_force_scalar<double>(double r2, double eps24, double sig2) {
  const double ir2 = rcp_nr<double>(r2);
  const double s2 = sig2 * ir2;
  const double s6 = s2 * s2 * s2;
  return (eps24 * ir2) * (s6 * fma(2.0, s6, -1.0));
}
// 1 / r2 to FP64 accuracy: FP32 path starts from the FP32 hardware reciprocal (recomputed; the
// compiler merges it with the one in lj_force_scalar) and takes one FP64 Newton step (2^-23 ->
// ~2^-46 relative); FP64 path uses the twice-refined FP64 reciprocal.
template <typename R> __device__ __forceinline__ double rcp_fp64_from(double r2);
template <> __device__ __forceinline__ double rcp_fp64_from<float>(double r2) {
  double r = (double)__builtin_amdgcn_rcpf((float)r2);
  const double e = fma(-r2, r, 1.0);
  return fma(r, e, r);
}
template <> __device__ __forceinline__ double rcp_fp64_from<double>(double r2) { return rcp_nr<double>(r2); }

// floor(a / b) for 0 <= a < 2^21 and b >= 1 from rb = the FP32 hardware reciprocal of b (1 ulp):
// (a + 1/2) / b lies at least 1/(2b) from an integer, while the FP32 result is within a relative
// 2^-22 of it, i.e. within (a + 1/2) 2^-22 / b < 1/(2b).
__device__ __forceinline__ int div_small(int a, float rb) { return (int)(((float)a + 0.5f) * rb); }

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// ---------------------------------------------------------------- exact order-free sums
// FP64 values summed in LDS as 64-bit integers, so that the result does not depend on the order in
// which concurrent lanes add (the j-side sums of the half-shell pair kernel).  x (|x| < 2^50) is
// split into h = round(x) and the residual x - h (exact, |x - h| <= 1/2), which is scaled by 2^50
// and rounded: absolute resolution 2^-51.  Adding the constant M = 1.5 2^52 to a value v with
// |v| < 2^51 leaves M + round(v) in FP64, whose bit pattern is that of M plus round(v): the raw
// patterns are summed and the count of terms times the pattern of M is subtracted at the end.
constexpr double FX_MAGIC = 6755399441055744.0;  // 1.5 * 2^52

__device__ __forceinline__ bool fx_add(unsigned long long *hi, unsigned long long *lo, double x) {
  const double a = x + FX_MAGIC;
  const double h = a - FX_MAGIC;
  const double b = fma(x - h, 0x1p50, FX_MAGIC);
  atomicAdd(hi, (unsigned long long)__double_as_longlong(a));
  atomicAdd(lo, (unsigned long long)__double_as_longlong(b));
  return fabs(x) < 0x1p50;  // false also for NaN
}

// Single-word variant for FP32-accurate terms: x scaled by 2^26 and rounded (absolute resolution
// 2^-27, |x| < 2^24).
__device__ __forceinline__ bool fx1_add(unsigned long long *w, double x) {
  atomicAdd(w, (unsigned long long)__double_as_longlong(fma(x, 0x1p26, FX_MAGIC)));
  return fabs(x) < 0x1p24;  // false also for NaN
}

__device__ __forceinline__ double fx1_value(unsigned long long w, unsigned k) {
  const unsigned long long m = (unsigned long long)__double_as_longlong(FX_MAGIC) * (unsigned long long)k;
  return (double)(long long)(w - m) * 0x1p-26;
}

// Variant for FP64 terms with a 32-bit high word: round(x) is the low half of the bit pattern of
// x + M, added to the int32 word hi (|x| < 2^23, so 256 terms cannot overflow it); the residual
// goes to lo as in fx_add.  12 bytes of LDS per value instead of 16.
__device__ __forceinline__ bool fx2_add(unsigned long long *lo, int *hi, double x) {
  const double a = x + FX_MAGIC;
  const double h = a - FX_MAGIC;
  atomicAdd(hi, (int)(unsigned)__double_as_longlong(a));
  atomicAdd(lo, (unsigned long long)__double_as_longlong(fma(x - h, 0x1p50, FX_MAGIC)));
  return fabs(x) < 0x1p23;  // false also for NaN
}

__device__ __forceinline__ double fx2_value(unsigned long long lo, int hi, unsigned k) {
  const unsigned long long m = (unsigned long long)__double_as_longlong(FX_MAGIC) * (unsigned long long)k;
  return (double)hi + (double)(long long)(lo - m) * 0x1p-50;
}

// The value of k terms added with fx_add.
__device__ __forceinline__ double fx_value(unsigned long long hi, unsigned long long lo, unsigned k) {
  const unsigned long long m = (unsigned long long)__double_as_longlong(FX_MAGIC) * (unsigned long long)k;
  return (double)(long long)(hi - m) + (double)(long long)(lo - m) * 0x1p-50;
}

// ---------------------------------------------------------------- neighbour-cell table
struct NbTable {
  int off[28];   // exclusive prefix of the 27 cell counts (off[27] = total staged)
  int start[27]; // first sorted slot of each neighbour cell
  double sh[27][3];
};

// Stencil entry k = 0..26 is (dx, dy, dz) = (k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1); entry 13
// is the home cell.  A neighbour index that leaves the grid wraps around, and the molecules of
// the wrapped cell are seen through the image shift -L (from below) or +L (from above).
// HALF (Newton's third law): only entries 13..26, stored as k = 0..13 -- the home cell first,
// then the 13 offsets that follow (0, 0, 0) in (dz, dy, dx) order.  Of two cells at opposite
// offsets exactly one lists the other, so every unordered pair of a cell and a periodic image of
// a neighbour is visited once; off[14..27] hold the total.
template <bool HALF = false>
__device__ __forceinline__ void build_nb(const CellsDev &c, int cell, NbTable &t) {
  constexpr int NE = HALF ? 14 : 27, E0 = HALF ? 13 : 0;
  const int lane = threadIdx.x;
  int cnt = 0;
  if (lane < NE) {
    const int e = lane + E0;
    const int cx = cell % c.nx, cy = (cell / c.nx) % c.ny, cz = cell / (c.nx * c.ny);
    int x = cx + e % 3 - 1, y = cy + (e / 3) % 3 - 1, z = cz + e / 9 - 1;
    double shx = 0.0, shy = 0.0, shz = 0.0;
    if (x < 0) x += c.nx, shx = -c.Lx;
    else if (x >= c.nx) x -= c.nx, shx = c.Lx;
    if (y < 0) y += c.ny, shy = -c.Ly;
    else if (y >= c.ny) y -= c.ny, shy = c.Ly;
    if (z < 0) z += c.nz, shz = -c.Lz;
    else if (z >= c.nz) z -= c.nz, shz = c.Lz;
    const int nc = (z * c.ny + y) * c.nx + x;
    const int s = c.cell_start[nc];
    cnt = c.cell_start[nc + 1] - s;
    t.start[lane] = s;
    t.sh[lane][0] = shx;
    t.sh[lane][1] = shy;
    t.sh[lane][2] = shz;
  }
  const int incl = wave_incl_scan(cnt);
  if (lane < NE) t.off[lane] = incl - cnt;
  const int tot = __shfl(incl, NE - 1, 64);
  if (lane >= NE && lane < 28) t.off[lane] = tot;
}

// Last stencil entry k with off[k] <= g (skips empty cells).
__device__ __forceinline__ int find_nb(const int *off, int g) {
  int lo = 0, hi = 27;
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Energy per unit moment product of one electrostatic site pair and its partial derivatives
// with respect to r and the cosines c_i = e_a.rhat, c_j = e_b.rhat, c_ij = e_a.e_b (rhat points
// from site b of molecule j to site a of molecule i).  ir = 1/r; krc3 = kappa / r_c^3.
// Per unit moment product: energy t (t0: the same without the reaction-field term) and its
// partial derivatives with respect to r, c_i, c_j and c_ij; ang is t0 / r^-n, the angular factor
// of the energy, with n = unit_rpow<KA, KB>().
template <typename R> struct Unit {
  R t, tr, ti, tj, tij, t0, ang;
};

template <int KA, int KB> constexpr int unit_rpow() {
  return 1 + (KA == KIND_CHG ? 0 : (KA == KIND_DIP ? 1 : 2)) + (KB == KIND_CHG ? 0 : (KB == KIND_DIP ? 1 : 2));
}

template <int KA, int KB, typename R>
__device__ __forceinline__ Unit<R> unit_terms(R ir, R ci, R cj, R cij, R krc3) {
#pragma clang fp contract(fast)  // products and sums fused where the compiler can (pair algebra only)
  Unit<R> u{0, 0, 0, 0, 0, 0, 0};
  const R ir2 = ir * ir, ir3 = ir2 * ir, ir4 = ir3 * ir;
  if constexpr (KA == KIND_CHG && KB == KIND_CHG) {
    u.ang = (R)1;
    u.t = ir;
    u.tr = -ir2;
  } else if constexpr (KA == KIND_CHG && KB == KIND_DIP) {
    u.ang = cj;
    u.t = cj * ir2;
    u.tr = (R)-2 * cj * ir3;
    u.tj = ir2;
  } else if constexpr (KA == KIND_DIP && KB == KIND_CHG) {
    u.ang = -ci;
    u.t = -ci * ir2;
    u.tr = (R)2 * ci * ir3;
    u.ti = -ir2;
  } else if constexpr (KA == KIND_CHG && KB == KIND_QUAD) {
    u.ang = (R)0.5 * fma((R)3 * cj, cj, (R)-1);
    u.t = u.ang * ir3;
    u.tr = (R)-3 * u.t * ir;
    u.tj = (R)3 * cj * ir3;
  } else if constexpr (KA == KIND_QUAD && KB == KIND_CHG) {
    u.ang = (R)0.5 * fma((R)3 * ci, ci, (R)-1);
    u.t = u.ang * ir3;
    u.tr = (R)-3 * u.t * ir;
    u.ti = (R)3 * ci * ir3;
  } else if constexpr (KA == KIND_DIP && KB == KIND_DIP) {
    const R g = fma((R)-3 * ci, cj, cij);
    u.ang = g;
    u.t0 = g * ir3;
    u.t = fma(g, ir3, -krc3 * cij);
    u.tr = (R)-3 * g * ir4;
    u.ti = (R)-3 * cj * ir3;
    u.tj = (R)-3 * ci * ir3;
    u.tij = ir3 - krc3;
  } else if constexpr (KA == KIND_DIP && KB == KIND_QUAD) {
    const R p = (R)1.5 * ir4;
    R g;
    {
#pragma clang fp contract(off)  // the angular factor of the energy keeps its unfused rounding
      g = ci - (R)5 * ci * cj * cj + (R)2 * cj * cij;
    }
    u.ang = (R)1.5 * g;
    u.t = p * g;
    u.tr = (R)-4 * u.t * ir;
    u.ti = p * fma((R)-5 * cj, cj, (R)1);
    u.tj = p * fma((R)-10 * ci, cj, (R)2 * cij);
    u.tij = p * (R)2 * cj;
  } else if constexpr (KA == KIND_QUAD && KB == KIND_DIP) {
    const R p = (R)-1.5 * ir4;
    R g;
    {
#pragma clang fp contract(off)
      g = cj - (R)5 * cj * ci * ci + (R)2 * ci * cij;
    }
    u.ang = (R)-1.5 * g;
    u.t = p * g;
    u.tr = (R)-4 * u.t * ir;
    u.tj = p * fma((R)-5 * ci, ci, (R)1);
    u.ti = p * fma((R)-10 * ci, cj, (R)2 * cij);
    u.tij = p * (R)2 * ci;
  } else {  // QUAD-QUAD
    const R p = (R)0.75 * ir4 * ir;
    const R s = fma((R)-5 * ci, cj, cij);
    const R ci2 = ci * ci, cj2 = cj * cj;
    R g;
    {
#pragma clang fp contract(off)
      g = (R)1 - (R)5 * ci2 - (R)5 * cj2 - (R)15 * ci2 * cj2 + (R)2 * s * s;
    }
    u.ang = (R)0.75 * g;
    u.t = p * g;
    u.tr = (R)-5 * u.t * ir;
    u.ti = p * ((R)-10 * ci - (R)30 * ci * cj2 - (R)20 * cj * s);
    u.tj = p * ((R)-10 * cj - (R)30 * cj * ci2 - (R)20 * ci * s);
    u.tij = p * (R)4 * s;
  }
  if constexpr (!(KA == KIND_DIP && KB == KIND_DIP)) u.t0 = u.t;
  return u;
}

// Slot layout of the per-molecule vectors for shape (SL, SC, SD, SQ).
template <int SL, int SC, int SD, int SQ> struct Slots {
  static constexpr int lj = 0, chg = SL, dip = SL + SC, dipax = SL + SC + SD, quad = SL + SC + 2 * SD,
                       quadax = SL + SC + 2 * SD + SQ, nv = SL + SC + 2 * SD + 2 * SQ;
};

}  // namespace mdcell
