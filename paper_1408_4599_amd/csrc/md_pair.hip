// Linked-cell pair kernels: forces, torques, energy and virial of rigid multi-centre molecules
// (Sec. 2 interaction models; Sec. 3 linked cells, periodic boundaries, summation of forces and
// torques per molecule).
//
// Work decomposition (details above each kernel):
//   * the cells around each home cell (edge >= r_c, so every partner inside the cutoff is there,
//     Sec. 3) are staged into LDS with their periodic image shift already applied, shared by the
//     wavefronts of a block (several home cells, or several wavefronts per dense cell): all 27
//     for single-site LJ, the home cell and its 13 forward neighbours (half shell) for
//     multi-site molecules;
//   * the lanes of a wavefront are n molecules x NS = min(8, floor(64 / n)) partner slices, and
//     lane (i, s) scans staged partners s, s + NS, ...;
//   * pass 1 lists the candidates inside the COM cutoff and pass 2 evaluates the listed pairs
//     only; the decision is always the exact FP64 test fma(dz, dz, fma(dy, dy, dx * dx)) < r_c^2
//     on d = r_i - (r_j + shift), so the set of interacting pairs is the brute-force set bit for
//     bit (the single-site FP32 path lists with an FP32 test whose threshold carries a proven
//     rounding guard band and re-tests the listed pairs exactly in FP64);
//   * the FP32 path (R = float) seeds reciprocals in FP32 and evaluates the single-site LJ force
//     scalar and the multipole forces and torques in FP32; separations of LJ sites, the
//     multi-site LJ terms (which share the energy's FP64 powers), pair energies (multipole
//     cosines and angular factors included) and all sums are FP64;
//   * slices are combined in a fixed order; every block writes one row of partials (energy,
//     virial diagonal, pair count) which a deterministic two-stage reduction sums in order.
// Single-site LJ pairs are evaluated from both ends (full shell): no partner sums at all.
// Multi-site pairs are evaluated once (Newton's third law, Fig. 1); the partner's terms are summed
// as exact integers in LDS, written to per-molecule rows and added in a fixed order by a gather,
// so results are bitwise reproducible either way.  The pair work is VALU-bound (no dense
// contraction: no MFMA).

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "md_device.h"

namespace mdcell {
namespace {

// ---------------------------------------------------------------- block partials
__device__ __forceinline__ void write_partial(double *partial, double u, double wx, double wy, double wz, double n) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    u += __shfl_xor(u, o);
    wx += __shfl_xor(wx, o);
    wy += __shfl_xor(wy, o);
    wz += __shfl_xor(wz, o);
    n += __shfl_xor(n, o);
  }
  if (threadIdx.x == 0) {
    double *p = partial + (int64_t)blockIdx.x * PARTIAL_COLS;
    p[0] = u, p[1] = wx, p[2] = wy, p[3] = wz, p[4] = n;
  }
}

// =====================================================================================
// Single-site Lennard-Jones (LJ or LJTS, Sec. 2): the molecule is its one site.
// =====================================================================================

// One LJ pair seen from molecule i: FP64 separation d (exact), r2 its squared length.
template <typename R> struct LJAcc {
  double fx = 0, fy = 0, fz = 0, u = 0, wx = 0, wy = 0, wz = 0;
  int n = 0;
  __device__ __forceinline__ void add(double dx, double dy, double dz, double r2, R eps24, R sig2, double eps4d,
                                      double sig2d) {
    // force scalar in R; products with the exact FP64 separation and all sums in FP64
    const double fs = lj_force_scalar<R>(r2, eps24, sig2);
    const double gx = fs * dx, gy = fs * dy, gz = fs * dz;
    fx += gx, fy += gy, fz += gz;
    wx = fma(gx, dx, wx), wy = fma(gy, dy, wy), wz = fma(gz, dz, wz);
    // pair energy in FP64 from the reciprocal refined to FP64 accuracy (LJTS shift added per count)
    const double ir2 = rcp_fp64_from<R>(r2);
    const double s2 = sig2d * ir2;
    const double s6 = s2 * s2 * s2;
    u = fma(eps4d * s6, s6 - 1.0, u);
    n += 1;
  }
};

// Path for a home cell with more than 64 molecules: lanes of wave 0 are split into NI molecule
// lanes x NS partner slices over the 27 cells, staged through LDS in chunks of CAP, every staged
// partner tested, 64 home molecules at a time.  Every thread of the block must call it (it
// synchronises the block).
template <typename R>
__device__ void lj1_cell_chunked(const CellsDev &c, const LJPair &p, double rc2, const PairOut &o, int cell,
                                 double *jx, double *jy, double *jz, const int CAP, NbTable &nb, double acc5[5]) {
  const int tid = threadIdx.x, lane = tid & 63;
  const bool w0 = tid < 64;
  const int hs = c.cell_start[cell], hn = c.cell_start[cell + 1] - hs;
  if (hn == 0) return;
  __syncthreads();
  if (w0) build_nb(c, cell, nb);
  __syncthreads();
  const int M = nb.off[27];
  const int self0 = nb.off[13];
  const int NI = hn <= 16 ? 16 : (hn <= 32 ? 32 : 64);
  const int NS = 64 / NI;
  const int il = lane & (NI - 1), sl = lane / NI;
  const R eps24 = (R)p.eps24, sig2 = (R)p.sig2;
  for (int ic = 0; ic < hn; ic += 64) {
    const int iloc = ic + il;
    const bool act = w0 && iloc < hn;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (act) xi = c.sx[hs + iloc], yi = c.sy[hs + iloc], zi = c.sz[hs + iloc];
    LJAcc<R> a;
    for (int jc = 0; jc < M; jc += CAP) {
      const int mj = min(CAP, M - jc);
      __syncthreads();
      for (int t = tid; t < mj; t += blockDim.x) {
        const int g = jc + t;
        const int k = find_nb(nb.off, g);
        const int src = nb.start[k] + (g - nb.off[k]);
        jx[t] = c.sx[src] + nb.sh[k][0];
        jy[t] = c.sy[src] + nb.sh[k][1];
        jz[t] = c.sz[src] + nb.sh[k][2];
      }
      __syncthreads();
      if (act) {
        const int self = self0 + iloc - jc;
        for (int t = sl; t < mj; t += NS) {
          const double dx = xi - jx[t], dy = yi - jy[t], dz = zi - jz[t];
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          if (r2 < rc2 && t != self) a.add(dx, dy, dz, r2, eps24, sig2, p.eps4, p.sig2);
        }
      }
    }
    if (w0) {
#pragma unroll
      for (int off = 16; off < 64; off <<= 1) {
        if (off >= NI) {
          a.fx += __shfl_xor(a.fx, off), a.fy += __shfl_xor(a.fy, off), a.fz += __shfl_xor(a.fz, off);
          a.u += __shfl_xor(a.u, off);
          a.wx += __shfl_xor(a.wx, off), a.wy += __shfl_xor(a.wy, off), a.wz += __shfl_xor(a.wz, off);
          a.n += __shfl_xor(a.n, off);
        }
      }
    }
    if (act && sl == 0) {
      const int64_t orig = c.perm[hs + iloc];  // 64-bit: 3 orig exceeds 2^31 beyond 7e8 molecules
      a.u -= (double)a.n * p.shift;
      o.force[3 * orig] = a.fx, o.force[3 * orig + 1] = a.fy, o.force[3 * orig + 2] = a.fz;
      if (o.torque) o.torque[3 * orig] = 0.0, o.torque[3 * orig + 1] = 0.0, o.torque[3 * orig + 2] = 0.0;
      if (o.u_mol) o.u_mol[orig] = 0.5 * a.u;
      if (o.w_mol) o.w_mol[orig] = 0.5 * (a.wx + a.wy + a.wz);
      if (o.nnb_mol) o.nnb_mol[orig] = a.n;
      acc5[0] += 0.5 * a.u, acc5[1] += 0.5 * a.wx, acc5[2] += 0.5 * a.wy, acc5[3] += 0.5 * a.wz;
      acc5[4] += (double)a.n;
    }
  }
}

// Fixed-order block reduction of the five partial columns (wave shuffles, then waves in order).
template <int NW>
__device__ __forceinline__ void write_partial_block(double *partial, double acc5[5], double (*red)[5],
                                                    int64_t row = -1) {
  if (row < 0) row = blockIdx.x;
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc5[q] += __shfl_xor(acc5[q], o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (NW == 1) {
    if (lane == 0) {
      double *pp = partial + row * PARTIAL_COLS;
      for (int q = 0; q < 5; ++q) pp[q] = acc5[q];
    }
    return;
  }
  if (lane == 0)
    for (int q = 0; q < 5; ++q) red[wave][q] = acc5[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double *pp = partial + row * PARTIAL_COLS;
    for (int q = 0; q < 5; ++q) {
      double v = red[0][q];
      for (int w = 1; w < NW; ++w) v += red[w][q];
      pp[q] = v;
    }
  }
}

// Single-site kernel with compaction.  A block of four wavefronts takes 1 x 2 x 2 home cells (one in
// x, two in y, two in z); their 27-cell neighbourhoods together span 3 x 4 x 4 cells, which are
// staged once into LDS (image shifts applied) in x-fastest order.  In that order a wavefront's
// stencil is three contiguous segments of nine cells (3 in x by 3 in y, one segment per z-layer).
// In a wavefront with n home molecules, lane l < n NS (NS = min(8, floor(64 / n))) takes molecule
// l % n and, in each segment, candidates s, s + NS, ... with s = l / n: all molecule lanes of a
// slice read the same partner, so LDS reads broadcast.
//
// Pass 1 (cutoff test) appends the staged slot of every hit to a per-lane list in LDS.
//   * FP64 path: the exact test fma(dz, dz, fma(dy, dy, dx * dx)) < r_c^2 on FP64 separations.
//   * FP32 path: each staged entry also holds x~ = fl32(x - o) relative to the tile centre o and
//     n~ = fl32(|x~|^2); the test is T = fma(-2 z~_i, z~_j, fma(-2 y~_i, y~_j, fma(-2 x~_i, x~_j,
//     n~_j))) < fl32(thr - n~_i), i.e. |x~_i - x~_j|^2 < thr, three FMAs per candidate.  thr
//     exceeds r_c^2 by a proven bound on the FP32 rounding (lj_guard_threshold), so the listed
//     pairs are a superset of the pairs inside the cutoff; pass 2 takes the exact FP64 decision.
// Pass 2 (when a list could overflow, and at the end): the lanes of each molecule copy their lists
// into one list per molecule (slices in order), then lane (i, s) evaluates its entries s, s + NS,
// ... in order: the molecule's hits split evenly over its lanes.  Each pair is evaluated from the
// exact FP64 separation (staged FP64 positions): the energy always in FP64 (from the FP32
// reciprocal refined by one FP64 Newton step on the FP32 path), the force scalar, force and
// virial in R.  FP32 sums of one flush are promoted to the lane's FP64 sums at its end.
// A block whose tile exceeds the LDS capacity walks the same candidates in the same order through
// per-wavefront windows of its segments: the same pairs, each evaluated the same way; only the
// points where lists are flushed can differ (a window change flushes), which regroups each
// molecule's sum over its lanes: a difference of rounding.  Slice sums are combined through LDS in
// a fixed order.  Home cells with more than 64 molecules use lj1_cell_chunked (a decision fixed by
// the configuration, not by the capacity).
constexpr int QCELLS = 48;  // 3 x 4 x 4 staged cells
constexpr int NSMAX = 8;
constexpr int SLACK = 32;  // spare tile entries read (never counted) past the end of a walk
constexpr int FLUSH_H = 3;  // listed partners per flush iteration in the 4-wave instances
constexpr unsigned short LIST_END = 0xFFFF;  // end marker of a hit list (slots stay below 4096)
typedef float f4v __attribute__((ext_vector_type(4)));

// LJ constants of the single-site kernels: FP64 model values, their FP32 roundings for the FP32
// force scalar, and the FP32 pass-1 threshold.
struct LJK {
  double eps4, eps24, sig2, shift, rc2;
  float eps24f, sig2f, thr;
};

// Sums of one flush of one lane: force and virial diagonal in R, energy in FP64, partner count.
template <typename R> struct LJFlush {
  R fx = 0, fy = 0, fz = 0, wx = 0, wy = 0, wz = 0;
  double u = 0.0;
  int n = 0;
};

// One listed partner at the exact FP64 separation d.
template <typename R>
__device__ __forceinline__ void lj_hit(LJFlush<R> &a, double dx, double dy, double dz, const LJK &k) {
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  if constexpr (std::is_same<R, float>::value) {
    if (!(r2 < k.rc2)) return;  // listed by the FP32 test, outside the exact cutoff
    const float y = __builtin_amdgcn_rcpf((float)r2);
    // energy: 1/r^2 refined to FP64 accuracy by one FP64 Newton step from the FP32 seed
    const double yd = fma((double)y, fma(-r2, (double)y, 1.0), (double)y);
    const double s2 = k.sig2 * yd, s6 = s2 * s2 * s2;
    a.u = fma(k.eps4 * s6, s6 - 1.0, a.u);
    // force scalar from the FP32 seed (1 ulp), force and virial in FP32
    const float t2 = k.sig2f * y, t6 = t2 * t2 * t2;
    const float fs = (k.eps24f * y) * (t6 * fmaf(2.0f, t6, -1.0f));
    const float ex = (float)dx, ey = (float)dy, ez = (float)dz;
    const float gx = fs * ex, gy = fs * ey, gz = fs * ez;
    a.fx += gx, a.fy += gy, a.fz += gz;
    a.wx = fmaf(gx, ex, a.wx), a.wy = fmaf(gy, ey, a.wy), a.wz = fmaf(gz, ez, a.wz);
  } else {
    const double y = rcp_nr<double>(r2);
    const double s2 = k.sig2 * y, s6 = s2 * s2 * s2;
    a.u = fma(k.eps4 * s6, s6 - 1.0, a.u);
    const double fs = (k.eps24 * y) * (s6 * fma(2.0, s6, -1.0));
    const double gx = fs * dx, gy = fs * dy, gz = fs * dz;
    a.fx += gx, a.fy += gy, a.fz += gz;
    a.wx = fma(gx, dx, a.wx), a.wy = fma(gy, dy, a.wy), a.wz = fma(gz, dz, a.wz);
  }
  a.n += 1;
}

// H listed partners at once (H independent dependency chains for the latency-bound flush), added
// to the sums in listing order, so the sums equal those of H lj_hit calls bit for bit.  FP32 path:
// a partner outside the exact cutoff (listed by the guard band) adds nothing.
template <typename R, int H>
__device__ __forceinline__ void lj_hitn(LJFlush<R> &a, const double (&dx)[H], const double (&dy)[H],
                                        const double (&dz)[H], const LJK &k) {
  double r2[H];
#pragma unroll
  for (int h = 0; h < H; ++h) r2[h] = fma(dz[h], dz[h], fma(dy[h], dy[h], dx[h] * dx[h]));
  if constexpr (std::is_same<R, float>::value) {
    bool in[H];
    double s6[H];
    float gx[H], gy[H], gz[H], ex[H], ey[H], ez[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      in[h] = r2[h] < k.rc2;
      const float y = __builtin_amdgcn_rcpf((float)r2[h]);
      const double yd = fma((double)y, fma(-r2[h], (double)y, 1.0), (double)y);
      const double s2 = k.sig2 * yd;
      s6[h] = s2 * s2 * s2;
      const float t2 = k.sig2f * y, t6 = t2 * t2 * t2;
      const float fs = (k.eps24f * y) * (t6 * fmaf(2.0f, t6, -1.0f));
      ex[h] = (float)dx[h], ey[h] = (float)dy[h], ez[h] = (float)dz[h];
      gx[h] = fs * ex[h], gy[h] = fs * ey[h], gz[h] = fs * ez[h];
    }
#pragma unroll
    for (int h = 0; h < H; ++h)
      if (in[h]) {
        a.u = fma(k.eps4 * s6[h], s6[h] - 1.0, a.u);
        a.fx += gx[h], a.fy += gy[h], a.fz += gz[h];
        a.wx = fmaf(gx[h], ex[h], a.wx), a.wy = fmaf(gy[h], ey[h], a.wy), a.wz = fmaf(gz[h], ez[h], a.wz);
        a.n += 1;
      }
  } else {
    double s6[H], gx[H], gy[H], gz[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const double y = rcp_nr<double>(r2[h]);
      const double s2 = k.sig2 * y;
      s6[h] = s2 * s2 * s2;
      const double fs = (k.eps24 * y) * (s6[h] * fma(2.0, s6[h], -1.0));
      gx[h] = fs * dx[h], gy[h] = fs * dy[h], gz[h] = fs * dz[h];
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      a.u = fma(k.eps4 * s6[h], s6[h] - 1.0, a.u);
      a.fx += gx[h], a.fy += gy[h], a.fz += gz[h];
      a.wx = fma(gx[h], dx[h], a.wx), a.wy = fma(gy[h], dy[h], a.wy), a.wz = fma(gz[h], dz[h], a.wz);
    }
    a.n += H;
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SUB: half-edge cells.  The molecules of each cell come sorted by half-edge cell (lower z-half
// first), the tile is staged in the order (y row, z half-layer, x) and a home molecule in z-half b
// walks, in each of its three y rows, the five z half-layers [2 hz + b, 2 hz + b + 5) of the eight
// (tile z half-layers 2 hz .. 2 hz + 5 surround home cell hz): the sixth lies more than one cell
// edge (>= r_c) away along z, so none of its pairs is inside the cutoff.  Each lane's range starts
// at its molecule's half; the runs all lanes fill are walked unchecked, the rest bounds-checked.
// WPE: wavefronts per SIMD the register allocation must allow.  5 where the LDS of a block leaves
// room for 5 blocks per CU (sparse tiles): the flush then takes one hit per iteration, since more
// spill at that register count; 4 where LDS holds 4 blocks (dense tiles), with FLUSH_H hits per
// iteration of the flush.
template <typename R, bool SUB, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_pair_lj(CellsDev c, LJK k, PairOut o, int cap, int lcap) {
  constexpr bool F32 = std::is_same<R, float>::value;
  // staged groups: tile cells (3 x 4 x 4, cell u = ux + 3 uy + 12 uz), or with SUB the cell halves
  // in the order g = (uy * 8 + z half-layer) * 3 + ux
  constexpr int NG = SUB ? 2 * QCELLS : QCELLS;
  extern __shared__ double dyn[];
  // LDS: [FP32 tile: cap float4 (FP32 path)] [FP64 tile: cap x 3 doubles] [per-lane lists: 256 x
  // lcap]; list entries are staged slots (16 bit)
  f4v *const t32 = (f4v *)dyn;
  double *const t64 = dyn + (F32 ? 2 * cap : 0);
  __attribute__((address_space(3))) f4v *const l32 = (__attribute__((address_space(3))) f4v *)t32;
  __attribute__((address_space(3))) double *const l64 = (__attribute__((address_space(3))) double *)t64;
  unsigned short *const lists = (unsigned short *)(t64 + 3 * cap);
  // per group: first tile slot (qoff, plus the total), first sorted index (qstart), image shift
  // (qsh; SUB: packed as qcode, each axis shift / L + 1 in two bits)
  __shared__ int qoff[NG + 1], qstart[NG];
  __shared__ double qsh[SUB ? 1 : QCELLS][3];
  __shared__ int qcode[SUB ? NG : 1];
  __shared__ double red[4][5];
  // neighbour table of the chunked path, in the (then unused) list area
  NbTable &nb = *(NbTable *)lists;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nby = (c.ny + 1) >> 1, nbz = (c.nz + 1) >> 1;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  double acc5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (b < c.nx * nby * nbz) {
    const int bx = b % c.nx, by = (b / c.nx) % nby, bz = b / (c.nx * nby);
    // tile cell u = ux + 3 uy + 12 uz covers cell (bx - 1 + ux, 2 by - 1 + uy, 2 bz - 1 + uz)
    if (tid < 64) {
      int cnt = 0;
      int ux = 0, uy = 0, uz = 0, s0 = 0, s1 = 0, sm = 0, code = 0;
      double shx = 0.0, shy = 0.0, shz = 0.0;
      if (tid < QCELLS) {
        ux = tid % 3, uy = (tid / 3) % 4, uz = tid / 12;
        int x = bx - 1 + ux, y = 2 * by - 1 + uy, z = 2 * bz - 1 + uz;
        int kx = 1, ky = 1, kz = 1;
        if (x < 0) x += c.nx, shx = -c.Lx, kx = 0;
        else if (x >= c.nx) x -= c.nx, shx = c.Lx, kx = 2;
        if (y < 0) y += c.ny, shy = -c.Ly, ky = 0;
        else if (y >= c.ny) y -= c.ny, shy = c.Ly, ky = 2;
        if (z < 0) z += c.nz, shz = -c.Lz, kz = 0;
        else if (z >= c.nz) z -= c.nz, shz = c.Lz, kz = 2;
        code = kx | ky << 2 | kz << 4;
        const int cc = (z * c.ny + y) * c.nx + x;
        if constexpr (SUB) {
          s0 = c.sub_start[8 * cc], sm = c.sub_start[8 * cc + 4], s1 = c.sub_start[8 * cc + 8];
        } else {
          s0 = c.cell_start[cc];
          cnt = c.cell_start[cc + 1] - s0;
        }
      }
      if constexpr (SUB) {
        // the cell's lower and upper z-halves are groups g and g + 3; counts first, then the scan
        // over lane l's groups 2 l, 2 l + 1 (g order)
        const int g = (uy * 8 + 2 * uz) * 3 + ux;
        if (tid < QCELLS) {
          qoff[g] = sm - s0, qoff[g + 3] = s1 - sm;
          qstart[g] = s0, qstart[g + 3] = sm;
          qcode[g] = code, qcode[g + 3] = code;
        }
        wave_sync_lds();
        const int c0 = tid < QCELLS ? qoff[2 * tid] : 0, c1 = tid < QCELLS ? qoff[2 * tid + 1] : 0;
        wave_sync_lds();
        const int incl = wave_incl_scan(c0 + c1);
        if (tid < QCELLS) qoff[2 * tid] = incl - c0 - c1, qoff[2 * tid + 1] = incl - c1;
        if (tid == QCELLS - 1) qoff[NG] = incl;
      } else {
        if (tid < QCELLS) qstart[tid] = s0, qsh[tid][0] = shx, qsh[tid][1] = shy, qsh[tid][2] = shz;
        const int incl = wave_incl_scan(cnt);
        if (tid < QCELLS) qoff[tid] = incl - cnt;
        if (tid == QCELLS - 1) qoff[QCELLS] = incl;
      }
    }
    __syncthreads();
    const int U = qoff[NG];
    // tile centre: origin of the FP32 coordinates
    const double ox = (bx + 0.5) * c.hx, oy = (2 * by + 1) * c.hy, oz = (2 * bz + 1) * c.hz;
    // stage entry: FP64 shifted position (x, y, z) at slot e, FP32 centre-relative copy and norm
    auto put = [&](int e, double x, double y, double z) {
      t64[3 * e] = x, t64[3 * e + 1] = y, t64[3 * e + 2] = z;
      if constexpr (F32) {
        const float fx = (float)(x - ox), fy = (float)(y - oy), fz = (float)(z - oz);
        t32[e] = f4v{fx, fy, fz, fmaf(fz, fz, fmaf(fy, fy, fx * fx))};
      }
    };
    // image shift of group g (exact: 0 or +-L)
    auto shift = [&](int g, double &sx, double &sy, double &sz) {
      if constexpr (SUB) {
        const int q = qcode[g];
        sx = (double)((q & 3) - 1) * c.Lx, sy = (double)(((q >> 2) & 3) - 1) * c.Ly;
        sz = (double)((q >> 4) - 1) * c.Lz;
      } else {
        sx = qsh[g][0], sy = qsh[g][1], sz = qsh[g][2];
      }
    };
    auto stage = [&](int e, int src, int g) {
      double sx, sy, sz;
      shift(g, sx, sy, sz);
      put(e, c.sx[src] + sx, c.sy[src] + sy, c.sz[src] + sz);
    };
    // SUB: the group of tile slot e among groups [glo, glo + n), n <= 32 (the last one whose first
    // slot is <= e; empty groups are passed over)
    auto group_of = [&](int e, int glo, int n) {
      int g = glo;
#pragma unroll
      for (int st = 16; st > 0; st >>= 1)
        if (g + st < glo + n && qoff[g + st] <= e) g += st;
      return g;
    };
    // this wavefront's home cell: tile cell uh (unshifted, since it lies inside the box); SUB: its
    // halves are groups gh and gh + 3
    const int hy = wave & 1, hz = wave >> 1;
    const bool hvalid = 2 * by + hy < c.ny && 2 * bz + hz < c.nz;
    const int uh = 1 + 3 * (hy + 1) + 12 * (hz + 1);
    const int gh = ((hy + 1) * 8 + 2 * (hz + 1)) * 3 + 1;
    const int hlow = SUB ? qoff[gh + 1] - qoff[gh] : 0;  // molecules in the lower z-half
    const int hn = !hvalid ? 0
                   : SUB ? __builtin_amdgcn_readfirstlane(hlow + qoff[gh + 4] - qoff[gh + 3])
                         : __builtin_amdgcn_readfirstlane(qoff[uh + 1] - qoff[uh]);
    const int hs = SUB ? qstart[gh] : qstart[uh];
    if (!__syncthreads_or(hn > 64)) {
      // the walk reads up to 4 NS - 1 <= 31 entries past a segment (results discarded), so the
      // tile needs that much slack
      const bool tiled = U + SLACK <= cap;  // block-uniform
      const int orig32 = lane < hn ? c.perm[hs + lane] : 0;
      if (tiled && SUB) {
        // wave w stages y row w (groups 24 w .. 24 w + 23), the first 128 entries loaded before
        // any is stored
        const int gb = 24 * wave, e0 = qoff[gb], e1 = qoff[gb + 24];
        double vx[2], vy[2], vz[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int e = e0 + 64 * q + lane;
          if (e < e1) {
            const int g = group_of(e, gb, 24), src = qstart[g] + (e - qoff[g]);
            double sx, sy, sz;
            shift(g, sx, sy, sz);
            vx[q] = c.sx[src] + sx, vy[q] = c.sy[src] + sy, vz[q] = c.sz[src] + sz;
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (e0 + 64 * q + lane < e1) put(e0 + 64 * q + lane, vx[q], vy[q], vz[q]);
        for (int e = e0 + 128 + lane; e < e1; e += 64) {
          const int g = group_of(e, gb, 24);
          stage(e, qstart[g] + (e - qoff[g]), g);
        }
        __syncthreads();
      } else if (tiled) {
        // stage by x-rows of three cells (contiguous in the sorted arrays unless x wraps): wave w
        // takes rows w, w + 4, w + 8, w + 12, the first 64 entries of all four rows loaded
        // before any is stored (one round of global-load latency), longer rows after
        double vx[4], vy[4], vz[4];
        int dst[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = 3 * (wave + 4 * q);
          const int e = qoff[u] + lane;
          dst[q] = -1;
          if (e < qoff[u + 3]) {
            const int cc = e < qoff[u + 1] ? u : (e < qoff[u + 2] ? u + 1 : u + 2);
            const int src = qstart[cc] + (e - qoff[cc]);
            vx[q] = c.sx[src] + qsh[cc][0], vy[q] = c.sy[src] + qsh[cc][1], vz[q] = c.sz[src] + qsh[cc][2];
            dst[q] = e;
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (dst[q] >= 0) put(dst[q], vx[q], vy[q], vz[q]);
        for (int q = 0; q < 4; ++q) {
          const int u = 3 * (wave + 4 * q);
          for (int e = qoff[u] + 64 + lane; e < qoff[u + 3]; e += 64) {
            const int cc = e < qoff[u + 1] ? u : (e < qoff[u + 2] ? u + 1 : u + 2);
            stage(e, qstart[cc] + (e - qoff[cc]), cc);
          }
        }
        __syncthreads();
      }
      const float rhn = __builtin_amdgcn_rcpf((float)(hn > 0 ? hn : 1));
      const int NS = hn > 0 ? min(NSMAX, div_small(64, rhn)) : 1;
      const int sl = hn > 0 ? div_small(lane, rhn) : NS, il = hn > 0 ? lane - sl * hn : 0;
      const float r2ns = 0.5f * __builtin_amdgcn_rcpf((float)NS);  // 1/(2 NS)
      const bool act = sl < NS;
      // FP64 sums of this lane over all flushes
      double sfx = 0.0, sfy = 0.0, sfz = 0.0, su = 0.0, swx = 0.0, swy = 0.0, swz = 0.0;
      int sn = 0;
      if (hn > 0) {
        // tile slot of this lane's molecule; SUB: its z-half zb (lower half first in the cell)
        const int zb = SUB && il >= hlow ? 1 : 0;
        const int self = SUB ? qoff[gh + 3 * zb] + il - zb * hlow : qoff[uh] + il;
        // this lane's molecule: FP64 position, FP32 test operands (idle lanes: far away)
        double xi = 1e30, yi = 1e30, zi = 1e30;
        float ax = 0.0f, ay = 0.0f, az = 0.0f, thri = -1.0f;
        if (act) {
          if (tiled) xi = t64[3 * self], yi = t64[3 * self + 1], zi = t64[3 * self + 2];
          else xi = c.sx[hs + il], yi = c.sy[hs + il], zi = c.sz[hs + il];
          if constexpr (F32) {
            const float fx = (float)(xi - ox), fy = (float)(yi - oy), fz = (float)(zi - oz);
            ax = -2.0f * fx, ay = -2.0f * fy, az = -2.0f * fz;
            thri = k.thr - fmaf(fz, fz, fmaf(fy, fy, fx * fx));
          }
        }
        const double rc2 = k.rc2;
        unsigned short *const wlist = lists + (size_t)wave * 64 * lcap;
        // staged slots: the whole tile (slot = tile index) or this wavefront's window of cq
        // entries, of which the first C are staged at a time
        const int cq = (cap - SLACK) >> 2;
        const int C = div_small(cq - SLACK, r2ns) * (2 * NS);
        const int wb = tiled ? 0 : wave * cq;  // slot of window entry 0
        // this lane's hit list: entry k at mylist[64 k]; lp is the next free entry
        __attribute__((address_space(3))) unsigned short *const mylist =
            (__attribute__((address_space(3))) unsigned short *)wlist + lane;
        __attribute__((address_space(3))) unsigned short *lp = mylist;
        __attribute__((address_space(3))) unsigned short *const lplim = mylist + 64 * (lcap - 2);
        // pass 2: every lane evaluates its own list in order.  (Sharing each molecule's hits evenly
        // over its lanes, through the lists' lengths and end markers, measured slower: its
        // bookkeeping per flush and per hit costs more than the shorter longest list saves.)
        // FP64 path: one set of FP64 sums for the whole walk; FP32 path: FP32 sums per flush,
        // promoted to the lane's FP64 sums (cascaded summation)
        LJFlush<double> a64;
        auto flush = [&]() {
          const int cnt = (int)(lp - mylist) >> 6;
          if (act) {
            // WPE 4: FLUSH_H hits per iteration (independent chains), the rest one at a time
            auto run = [&](auto &acc) {
              using A = typename std::remove_reference<decltype(acc)>::type;
              using RA = decltype(A::fx);
              int q = 0;
              if constexpr (WPE <= 4) {
                constexpr int H = FLUSH_H;
                for (; q + H <= cnt; q += H) {
                  double dx[H], dy[H], dz[H];
#pragma unroll
                  for (int h = 0; h < H; ++h) {
                    const int e = mylist[64 * (q + h)];
                    dx[h] = xi - l64[3 * e], dy[h] = yi - l64[3 * e + 1], dz[h] = zi - l64[3 * e + 2];
                  }
                  lj_hitn<RA, H>(acc, dx, dy, dz, k);
                }
              }
              for (; q < cnt; ++q) {
                const int e = mylist[64 * q];
                lj_hit<RA>(acc, xi - l64[3 * e], yi - l64[3 * e + 1], zi - l64[3 * e + 2], k);
              }
            };
            if constexpr (F32) {
              LJFlush<float> a;
              run(a);
              sfx += (double)a.fx, sfy += (double)a.fy, sfz += (double)a.fz;
              swx += (double)a.wx, swy += (double)a.wy, swz += (double)a.wz;
              su += a.u, sn += a.n;
            } else {
              run(a64);
            }
          }
          lp = mylist;
        };
        const int sla = act ? sl : 0;  // idle lanes walk with slice 0
        // candidate pair (slots t, t + 1): FP32 test operands, or FP64 positions
        using V = typename std::conditional<F32, f4v, double>::type;
        struct Cand {
          V a0, a1, a2, b0, b1, b2;
        };
        auto load = [&](Cand &q, int t) {
          if constexpr (F32) {
            q.a0 = l32[t], q.b0 = l32[t + 1];
          } else {
            q.a0 = l64[3 * t], q.a1 = l64[3 * t + 1], q.a2 = l64[3 * t + 2];
            q.b0 = l64[3 * t + 3], q.b1 = l64[3 * t + 4], q.b2 = l64[3 * t + 5];
          }
        };
        // test the pair at slot t, list the hits (the slot is always written; the count advances
        // on a hit); lim: slots at or past it are not candidates (checked steps only)
        auto step = [&](const Cand &q, int t, int sself, int lim, auto tail, auto home) {
          bool ha, hb;
          if constexpr (F32) {
            ha = fmaf(az, q.a0.z, fmaf(ay, q.a0.y, fmaf(ax, q.a0.x, q.a0.w))) < thri;
            hb = fmaf(az, q.b0.z, fmaf(ay, q.b0.y, fmaf(ax, q.b0.x, q.b0.w))) < thri;
          } else {
            const double pax = xi - q.a0, pay = yi - q.a1, paz = zi - q.a2;
            const double pbx = xi - q.b0, pby = yi - q.b1, pbz = zi - q.b2;
            ha = fma(paz, paz, fma(pay, pay, pax * pax)) < rc2;
            hb = fma(pbz, pbz, fma(pby, pby, pbx * pbx)) < rc2;
          }
          if (tail) ha = ha && t < lim, hb = hb && t + 1 < lim;
          if (home) ha = ha && t != sself, hb = hb && t + 1 != sself;
          *lp = (unsigned short)t;
          lp += ha ? 64 : 0;
          *lp = (unsigned short)(t + 1);
          lp += hb ? 64 : 0;
          if (__any(lp > lplim)) flush();
        };
        // wave-uniform range [cs, ce) of tile indices, staged at slot = index - off: slice s tests
        // the adjacent slots 2 s, 2 s + 1 of every run of 2 NS candidates, two runs per trip with
        // the next run's pair loaded before the current one is tested.  The walk reads up to
        // 2 NS - 1 slots past the range (the tile keeps SLACK spare entries); only the last,
        // partial run is bounds-checked, and only the home layer holds the molecule itself.
        auto walk = [&](int cs, int ce, int off, auto home) {
          int sa = cs + 2 * sla - off;  // slot of this lane's first candidate
          const int send = ce - off, sself = self - off;
          Cand A, B;
          load(A, sa);
          int kb = cs;
          for (; kb + 4 * NS <= ce; kb += 4 * NS, sa += 4 * NS) {
            load(B, sa + 2 * NS);
            step(A, sa, sself, send, std::false_type(), home);
            load(A, sa + 4 * NS);
            step(B, sa + 2 * NS, sself, send, std::false_type(), home);
          }
          if (kb + 2 * NS <= ce) {
            step(A, sa, sself, send, std::false_type(), home);
            kb += 2 * NS, sa += 2 * NS;
            if (kb < ce) load(A, sa);
          }
          if (kb < ce) step(A, sa, sself, send, std::true_type(), home);
        };
        // SUB, whole tile staged: this lane's range [rs, re) of tile slots; the first nf runs are
        // full for every lane, the others up to nall are checked.  Loads are kept inside the tile
        // (a clamped load only feeds checked, uncounted candidates).
        auto walk_lane = [&](int rs, int re, int nf, int nall, auto home) {
          const int tlim = cap - 2;
          int sa = rs + 2 * sla;
          Cand A, B;
          load(A, min(sa, tlim));
          int j = 0;
          for (; j + 2 <= nf; j += 2, sa += 4 * NS) {
            load(B, sa + 2 * NS);
            step(A, sa, self, re, std::false_type(), home);
            load(A, min(sa + 4 * NS, tlim));
            step(B, sa + 2 * NS, self, re, std::false_type(), home);
          }
          if (j < nf) {
            step(A, sa, self, re, std::false_type(), home);
            ++j, sa += 2 * NS;
            load(A, min(sa, tlim));
          }
          for (; j < nall; ++j, sa += 2 * NS) {
            step(A, sa, self, re, std::true_type(), home);
            load(A, min(sa + 2 * NS, tlim));
          }
        };
        // one range of tile indices [lo, hi): walked at once when the whole tile is staged, else
        // through the window, [cs, ce) at a time, the previous window flushed first (lk: source
        // group of tile index e)
        auto segments = [&](int lo, int hi, auto lk, auto home) {
          for (int cs = lo, ce; cs < hi; cs = ce) {
            ce = tiled ? hi : min(hi, cs + C);
            const int off = tiled ? 0 : cs - wb;  // slot = tile index - off
            if (!tiled) {
              flush();
              for (int e = cs + lane; e < ce; e += 64) {
                const int g = lk(e);
                stage(e - off, qstart[g] + (e - qoff[g]), g);
              }
              wave_sync_lds();
            }
            walk(cs, ce, off, home);
          }
        };
        if constexpr (SUB) {
          // y rows hy .. hy + 2 of the tile; in row uy the groups of z half-layer 2 hz onwards start
          // at gy = 24 uy + 6 hz, a lane in z-half zb walks [qoff[gy + 3 zb], qoff[gy + 3 zb + 15])
          if (tiled) {
            for (int r = 0; r < 3; ++r) {
              const int gy = 24 * (hy + r) + 6 * hz;
              const int l0 = __builtin_amdgcn_readfirstlane(qoff[gy + 15] - qoff[gy]);
              const int l1 = __builtin_amdgcn_readfirstlane(qoff[gy + 18] - qoff[gy + 3]);
              const int rs = qoff[gy + 3 * zb], re = qoff[gy + 3 * zb + 15];
              const int nf = div_small(min(l0, l1), r2ns), nall = div_small(max(l0, l1) + 2 * NS - 1, r2ns);
              if (r == 1) walk_lane(rs, re, nf, nall, std::true_type());
              else walk_lane(rs, re, nf, nall, std::false_type());
            }
          } else {
            // the window holds uniform ranges: all six half-layers of each row, nothing culled
            for (int r = 0; r < 3; ++r) {
              const int gy = 24 * (hy + r) + 6 * hz;
              const int lo = __builtin_amdgcn_readfirstlane(qoff[gy]);
              const int hi = __builtin_amdgcn_readfirstlane(qoff[gy + 18]);
              auto lk = [&](int e) { return group_of(e, 24 * (hy + r), 24); };
              if (r == 1) segments(lo, hi, lk, std::true_type());
              else segments(lo, hi, lk, std::false_type());
            }
          }
        } else {
          for (int d = 0; d < 3; ++d) {
            const int u0 = 3 * hy + 12 * (hz + d);
            const int lo = __builtin_amdgcn_readfirstlane(qoff[u0]);
            const int hi = __builtin_amdgcn_readfirstlane(qoff[u0 + 9]);
            auto lk = [&](int e) {
              int u = u0;
              while (e >= qoff[u + 1]) ++u;
              return u;
            };
            if (d == 1) segments(lo, hi, lk, std::true_type());
            else segments(lo, hi, lk, std::false_type());
          }
        }
        flush();
        if constexpr (!F32) {
          sfx = a64.fx, sfy = a64.fy, sfz = a64.fz, swx = a64.wx, swy = a64.wy, swz = a64.wz;
          su = a64.u, sn = a64.n;
        }
      }
      // combine the slices of each molecule in a fixed order through LDS (the tile is free now)
      __syncthreads();
      double *sred = dyn + (size_t)wave * 64 * 8;
      if (act) {
        double *e = sred + lane;  // [quantity][lane]: consecutive lanes, distinct banks
        e[0] = sfx, e[64] = sfy, e[128] = sfz, e[192] = su, e[256] = swx, e[320] = swy, e[384] = swz;
        e[448] = (double)sn;
      }
      __syncthreads();
      if (lane < hn) {
        double v[8];
        for (int q = 0; q < 8; ++q) v[q] = sred[q * 64 + lane];
        for (int s = 1; s < NS; ++s)
          for (int q = 0; q < 8; ++q) v[q] += sred[q * 64 + lane + s * hn];
        const double nn = v[7];
        const double u = v[3] - nn * k.shift;
        const int64_t orig = orig32;  // 64-bit: 3 orig exceeds 2^31 beyond 7e8 molecules
        o.force[3 * orig] = v[0], o.force[3 * orig + 1] = v[1], o.force[3 * orig + 2] = v[2];
        if (o.torque) o.torque[3 * orig] = 0.0, o.torque[3 * orig + 1] = 0.0, o.torque[3 * orig + 2] = 0.0;
        if (o.u_mol) o.u_mol[orig] = 0.5 * u;
        if (o.w_mol) o.w_mol[orig] = 0.5 * (v[4] + v[5] + v[6]);
        if (o.nnb_mol) o.nnb_mol[orig] = (int)nn;
        acc5[0] = 0.5 * u, acc5[1] = 0.5 * v[4], acc5[2] = 0.5 * v[5], acc5[3] = 0.5 * v[6], acc5[4] = nn;
      }
    } else {
      const LJPair p{k.eps4, k.eps24, k.sig2, k.shift, 0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < 4; ++w) {
        const int fy = 2 * by + (w & 1), fz = 2 * bz + (w >> 1);
        if (fy < c.ny && fz < c.nz)
          lj1_cell_chunked<R>(c, p, k.rc2, o, (fz * c.ny + fy) * c.nx + bx, dyn, dyn + cap, dyn + 2 * cap, cap, nb,
                              acc5);
      }
    }
  }
  write_partial_block<4>(o.partial, acc5, red);
}

// Threshold of the FP32 cutoff test of k_pair_lj: every pair with (FP64) r^2 < r_c^2 passes
// T < fl32(thr - n~_i).  With u = 2^-24 and rho = (1.5 h_x, 2 h_y, 2 h_z) the largest offset of a
// staged position from the tile centre, R = |rho|:
//   * stored coordinates x~ = fl32(x - o) differ from x - o by at most u rho_k per axis, so the
//     FP32 separation a - b is within 2 u R of the exact one and |a - b|^2 <= r^2 + 4 u R r_c +
//     4 u^2 R^2 near the cutoff;
//   * n~ = fl32(|x~|^2) by two FMAs and a product: error <= 3.01 u R^2; the three FMAs of T round
//     partial sums of magnitude <= 3 R^2: error <= 9 u R^2; fl32(thr - n~_i) loses <= u (thr + R^2);
// so T < fl32(thr - n~_i) holds whenever thr (1 - u) > r_c^2 (1 + 2^-51) + 4 u R r_c + 16.02 u R^2 +
// 4 u^2 R^2.  thr = (r_c^2 + 4 u R r_c + 17 u R^2)(1 + 2 u), rounded up to FP32, satisfies it with
// margin; at r_c = 2.5, h = 2.54 it exceeds r_c^2 by 1.3e-5 relative, so pass 2 rejects about
// 1e-4 listed candidates per molecule.
inline float lj_guard_threshold(double rc, double hx, double hy, double hz) {
  const double u = 0x1p-24;
  const double R = std::sqrt(2.25 * hx * hx + 4.0 * hy * hy + 4.0 * hz * hz) * (1.0 + 1e-12);
  const double thr = (rc * rc + 4.0 * u * R * rc + 17.0 * u * R * R) * (1.0 + 2.0 * u);
  float t = (float)thr;
  if ((double)t < thr) t = std::nextafter(t, INFINITY);
  return t;
}

// Staged-partner capacity of the LJ tile: the 48 tile cells at 1.12 x the mean occupancy + 32,
// rounded up to 32, within [256, 4096]; denser tiles take the windowed walk.  (List entries are
// 16-bit staged slots.)
inline int lj1_tile_cap(int64_t N, int64_t ncell) {
  const double mean = (double)N / (double)ncell;
  int cap = (int)(QCELLS * mean * 1.12) + 32;
  cap = (cap + 31) / 32 * 32;
  return cap < 256 ? 256 : (cap > 4096 ? 4096 : cap);
}

// Per-lane hit-list length: the expected hits of a lane, h = (4/3 pi r_c^3 N/V) / NS, plus 2.5
// Poisson standard deviations and 2, so that most wavefronts evaluate their hits once, at the end;
// fuller lists are flushed early (pass 2) and restarted.
inline int lj1_list_cap(int64_t N, double V, double rc, int64_t ncell) {
  const double mean = (double)N / (double)ncell;
  int NS = (int)(64.0 / (mean > 1.0 ? mean : 1.0));
  NS = NS < 1 ? 1 : (NS > NSMAX ? NSMAX : NS);
  const double hits = 4.18879020478639 * rc * rc * rc * (double)N / V / NS;
  int l = (int)std::ceil(hits + 2.5 * std::sqrt(hits) + 2.0);
  l = (l + 3) / 4 * 4;
  return l < 16 ? 16 : (l > 64 ? 64 : l);
}

// =====================================================================================
// Multi-site molecules: LJ sites (Lorentz-Berthelot, optional shift) + point charges, point
// dipoles, linear point quadrupoles (k_C = 1) + reaction field on dipole pairs.
// =====================================================================================

template <typename R> __device__ __forceinline__ void cross_acc(R *T, const R *a, const R *f) {
#pragma clang fp contract(fast)
  T[0] += a[1] * f[2] - a[2] * f[1];
  T[1] += a[2] * f[0] - a[0] * f[2];
  T[2] += a[0] * f[1] - a[1] * f[0];
}

// Accumulators of one molecule pair (seen from molecule i).  The energy is summed in FP64 from
// FP64 parameters (mixed LJ parameters, moment products, the reaction-field factor), so that their
// rounding to R leaves no systematic error in U.
template <typename R> struct PairAcc {
  R F[3], T[3];
  double u;
};

// One electrostatic site pair: site a of i (offset oa, axis ea) and site b of j (ob, eb).
template <int KA, int KB, typename R>
__device__ __forceinline__ void elec_site(R pm, double pmd, const R *oa, const R *ea, const R *ob, const R *eb, R dx,
                                          R dy, R dz, double dxd, double dyd, double dzd, R krc3, double krc3d,
                                          PairAcc<R> &acc) {
#pragma clang fp contract(fast)
  const R rx = dx + oa[0] - ob[0], ry = dy + oa[1] - ob[1], rz = dz + oa[2] - ob[2];
  const R r2 = fma(rz, rz, fma(ry, ry, rx * rx));
  const R ir = rsq_nr<R>(r2);
  const R rh[3] = {rx * ir, ry * ir, rz * ir};
  const R ci = (KA != KIND_CHG) ? fma(ea[2], rh[2], fma(ea[1], rh[1], ea[0] * rh[0])) : (R)0;
  const R cj = (KB != KIND_CHG) ? fma(eb[2], rh[2], fma(eb[1], rh[1], eb[0] * rh[0])) : (R)0;
  const R cij = (KA != KIND_CHG && KB != KIND_CHG) ? fma(ea[2], eb[2], fma(ea[1], eb[1], ea[0] * eb[0])) : (R)0;
  const Unit<R> t = unit_terms<KA, KB, R>(ir, ci, cj, cij, krc3);
  R f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R g = t.tr * rh[k];
    if constexpr (KA != KIND_CHG) g += t.ti * (ea[k] - ci * rh[k]) * ir;
    if constexpr (KB != KIND_CHG) g += t.tj * (eb[k] - cj * rh[k]) * ir;
    f[k] = -pm * g;
  }
  acc.F[0] += f[0], acc.F[1] += f[1], acc.F[2] += f[2];
  cross_acc(acc.T, oa, f);
  if constexpr (KA != KIND_CHG) {
    R ga[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ga[k] = t.ti * rh[k];
      if constexpr (KB != KIND_CHG) ga[k] += t.tij * eb[k];
      ga[k] *= -pm;
    }
    cross_acc(acc.T, ea, ga);  // tau -= e_a x dU/de_a
  }
  // energy in FP64: the site separation from the FP64 COM separation (exact when both sites sit
  // at their centres), 1/r refined by one FP64 Newton step, and the cosines and angular factor in
  // FP64 from the stored axes
  double ue, cijd = (double)cij;
  if constexpr (sizeof(R) == 8) {
    ue = t.t0;
  } else {
    const double rxd = dxd + (double)(oa[0] - ob[0]), ryd = dyd + (double)(oa[1] - ob[1]);
    const double rzd = dzd + (double)(oa[2] - ob[2]);
    const double r2d = fma(rzd, rzd, fma(ryd, ryd, rxd * rxd));
    double y = (double)ir;
    y = y * fma(-0.5 * r2d, y * y, 1.5);
    double yn = y;
#pragma unroll
    for (int k = 1; k < unit_rpow<KA, KB>(); ++k) yn *= y;
    if constexpr (KA == KIND_CHG && KB == KIND_CHG) {
      ue = yn;
    } else {
      const double ead[3] = {(double)ea[0], (double)ea[1], (double)ea[2]};
      const double ebd[3] = {(double)eb[0], (double)eb[1], (double)eb[2]};
      const double cid = (KA != KIND_CHG) ? fma(ead[2], rzd, fma(ead[1], ryd, ead[0] * rxd)) * y : 0.0;
      const double cjd = (KB != KIND_CHG) ? fma(ebd[2], rzd, fma(ebd[1], ryd, ebd[0] * rxd)) * y : 0.0;
      if constexpr (KA != KIND_CHG && KB != KIND_CHG) cijd = fma(ead[2], ebd[2], fma(ead[1], ebd[1], ead[0] * ebd[0]));
      ue = unit_terms<KA, KB, double>(y, cid, cjd, cijd, krc3d).ang * yn;
    }
  }
  if constexpr (KA == KIND_DIP && KB == KIND_DIP) ue = fma(-krc3d, cijd, ue);
  acc.u = fma(pmd, ue, acc.u);
}

// All electrostatic site pairs of kinds (KA on i, KB on j).
// vi: all site vectors of i; vj: the electrostatic site vectors of j (slots from SL on).
template <int KA, int KB, int SL, int SC, int SD, int SQ, bool MIX, typename R>
__device__ __forceinline__ void elec_group(const CompDev &A, const CompDev &B, const R (*vi)[3], const R *vj,
                                           R dx, R dy, R dz, double dxd, double dyd, double dzd, R krc3,
                                           double krc3d, PairAcc<R> &acc) {
  using S = Slots<SL, SC, SD, SQ>;
  constexpr int NA = KA == KIND_CHG ? SC : (KA == KIND_DIP ? SD : SQ);
  constexpr int NB = KB == KIND_CHG ? SC : (KB == KIND_DIP ? SD : SQ);
  constexpr int OA = KA == KIND_CHG ? S::chg : (KA == KIND_DIP ? S::dip : S::quad);
  constexpr int OB = KB == KIND_CHG ? S::chg : (KB == KIND_DIP ? S::dip : S::quad);
  constexpr int EA = KA == KIND_DIP ? S::dipax : (KA == KIND_QUAD ? S::quadax : 0);
  constexpr int EB = KB == KIND_DIP ? S::dipax : (KB == KIND_QUAD ? S::quadax : 0);
  const int na = MIX ? (KA == KIND_CHG ? A.n_chg : (KA == KIND_DIP ? A.n_dip : A.n_quad)) : NA;
  const int nb = MIX ? (KB == KIND_CHG ? B.n_chg : (KB == KIND_DIP ? B.n_dip : B.n_quad)) : NB;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    if (a >= na) break;
    const double mad = KA == KIND_CHG ? A.chg_q[a] : (KA == KIND_DIP ? A.dip_mu[a] : A.quad_Q[a]);
    const R ma = (R)mad;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b >= nb) break;
      const double mbd = KB == KIND_CHG ? B.chg_q[b] : (KB == KIND_DIP ? B.dip_mu[b] : B.quad_Q[b]);
      elec_site<KA, KB, R>(ma * (R)mbd, mad * mbd, vi[OA + a], vi[EA + a], vj + 3 * (OB - SL + b),
                           vj + 3 * (EB - SL + b), dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
    }
  }
}

// One molecule pair seen from i: d = r_i - r_j (FP64, image shift applied).  LJ site separations,
// energies and force scalars are formed in FP64 from the FP64 site offsets (vil, vjl), from one
// 1/r^2 (FP32-seeded for R = float); all electrostatic terms are evaluated in R from the site
// vectors vi and vje (electrostatic slots of j).  gfx950 issues FP64 adds and fmas at the FP32
// rate, so only the reciprocals and the multipole polynomials gain from R = float.
template <int SL, int SC, int SD, int SQ, bool MIX, typename R>
__device__ __forceinline__ void mol_pair(const ModelDev *__restrict__ md, int ci, int cj, const double (*vil)[3],
                                         const R (*vi)[3], const double *vjl, const R *vje, double dxd, double dyd,
                                         double dzd, PairAcc<R> &acc) {
#pragma clang fp contract(fast)
  const CompDev &A = md->comp[ci];
  const CompDev &B = md->comp[cj];
  const int nla = MIX ? A.n_lj : SL, nlb = MIX ? B.n_lj : SL;
#pragma unroll
  for (int a = 0; a < SL; ++a) {
    if (a >= nla) break;
    const double ax = dxd + vil[a][0], ay = dyd + vil[a][1], az = dzd + vil[a][2];
    double fa[3] = {0.0, 0.0, 0.0};  // force on site a from all LJ sites of j (one lever-arm product)
#pragma unroll
    for (int b = 0; b < SL; ++b) {
      if (b >= nlb) break;
      const LJPair &p = md->lj[ci][cj][a][b];
      const double rx = ax - vjl[3 * b], ry = ay - vjl[3 * b + 1], rz = az - vjl[3 * b + 2];
      const double r2 = fma(rz, rz, fma(ry, ry, rx * rx));
      // 1/r^2 to FP64 accuracy (FP32 path: from the FP32 hardware reciprocal and one FP64 Newton
      // step), shared by the energy and the force scalar: FP64 arithmetic issues at the FP32 rate,
      // and one FP64 chain costs fewer instructions than an FP32 force chain plus conversions
      const double ir2d = rcp_fp64_from<R>(r2);
      const double s2d = p.sig2 * ir2d;
      const double s6d = s2d * s2d * s2d;
      acc.u = fma(p.eps4 * s6d, s6d - 1.0, acc.u);  // the shift is summed per molecule pair
      const double fs = (p.eps24 * ir2d) * (s6d * fma(2.0, s6d, -1.0));
      fa[0] = fma(fs, rx, fa[0]), fa[1] = fma(fs, ry, fa[1]), fa[2] = fma(fs, rz, fa[2]);
    }
    acc.F[0] += (R)fa[0], acc.F[1] += (R)fa[1], acc.F[2] += (R)fa[2];
    // its torque about the centre from the FP64 offset
    acc.T[0] += (R)(vil[a][1] * fa[2] - vil[a][2] * fa[1]);
    acc.T[1] += (R)(vil[a][2] * fa[0] - vil[a][0] * fa[2]);
    acc.T[2] += (R)(vil[a][0] * fa[1] - vil[a][1] * fa[0]);
  }
  const R dx = (R)dxd, dy = (R)dyd, dz = (R)dzd;
  const R *vj = vje;
  if constexpr (SC + SD + SQ > 0) {
    const double krc3d = md->kappa_rc3;
    const R krc3 = (R)krc3d;
    if constexpr (SC > 0) {
      elec_group<KIND_CHG, KIND_CHG, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
      if constexpr (SD > 0) {
        elec_group<KIND_CHG, KIND_DIP, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
        elec_group<KIND_DIP, KIND_CHG, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
      }
      if constexpr (SQ > 0) {
        elec_group<KIND_CHG, KIND_QUAD, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
        elec_group<KIND_QUAD, KIND_CHG, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
      }
    }
    if constexpr (SD > 0) {
      elec_group<KIND_DIP, KIND_DIP, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
      if constexpr (SQ > 0) {
        elec_group<KIND_DIP, KIND_QUAD, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
        elec_group<KIND_QUAD, KIND_DIP, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
      }
    }
    if constexpr (SQ > 0)
      elec_group<KIND_QUAD, KIND_QUAD, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, dxd, dyd, dzd, krc3, krc3d, acc);
  }
}

// One block of W wavefronts per home cell, half shell (Newton's third law, Fig. 1): the home cell
// and the 13 forward neighbours are staged through LDS in windows of CAP molecules shared by the
// block (COM position in FP64, LJ site offsets in FP64, electrostatic site vectors in R, component
// id; the COM alone for a single-site model), home cell first; home molecule i pairs with staged
// molecule g when g > i (every pair of the home cell once, every forward molecule).  The home molecules are split evenly over the
// wavefronts, and in a wavefront with n of them lanes are n molecules x NS partner slices
// (NS = min(8, floor(64 / n))).  Pass 1 runs the exact FP64 COM cutoff test and appends hits
// (window slots, one byte) to per-lane lists; pass 2 evaluates the listed molecule pairs, the hits
// of each molecule (its NS lanes' lists in slice order) split into NS contiguous equal parts.
// The molecule's own sums stay in registers (FP64, slices combined in a fixed order) and go to row
// 0.  The partner receives -F and -tau - d x F (the pair energy is invariant under a rigid
// rotation of both molecules, so the torques about the two centres and d x F sum to zero), plus
// half of the pair energy and virial when asked for; these go to per-slot LDS sums in exact
// integer arithmetic (fx1_add on the FP32 path, fx2_add on the FP64 path, fx_add for u, w), which
// the block writes, once per window, to the partner's row 1 + k (k its half-stencil entry).  Each (row, molecule) is written by exactly one block, also
// when its home cell is empty.  A home cell with more than 64 W molecules is taken 64 W at a time;
// later rounds add to the rows of the first.
template <typename R, int SL, int SC, int SD, int SQ, bool MIX, int CAP, int W, int WPE>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE))) void k_pair_ms(CellsDev c, const ModelDev *__restrict__ md,
                                                                                     double rc2, PairOut o) {
  constexpr int NV = Slots<SL, SC, SD, SQ>::nv;
  constexpr int NE = NV - SL > 0 ? NV - SL : 1;  // electrostatic slots
  constexpr int LCAP = 32;
  static_assert(CAP <= 256, "list entries are bytes");
  __shared__ double jp[CAP * 3 + 48];  // slack: the walk reads up to 2 NS - 1 slots past the window
  constexpr int CAPV = SL == 1 && NV == 1 && !MIX ? 1 : CAP;  // no site vectors for a centre-only site
  __shared__ double jl[CAPV][SL * 3];  // LJ site offsets (FP64)
  __shared__ R jv[CAPV][NE * 3];       // electrostatic site offsets and axes
  __shared__ int jc_[MIX ? CAP : 1];
  __shared__ unsigned char lists[W][LCAP * 64];
  __shared__ int scnts[W][64];
  __shared__ NbTable nb;
  __shared__ double red[W][5];
  __shared__ unsigned jn[CAP];  // partner terms per slot
  __shared__ int jbad[CAP];     // a term of the slot was out of the fixed-point range
  // partner sums [words][CAP]: force (and torque) components one 64-bit word each (R = float:
  // fx1_add; R = double: the low words of fx2_add), then u and w two words each (fx_add) when
  // asked for; for R = double the 32-bit high words of the force (and torque) follow, [NT][CAP]
  extern __shared__ unsigned long long jacc[];
  constexpr bool F64 = sizeof(R) == 8;
  // one LJ site at the centre (single-site model): no site vectors, no torques, NT = 3 partner
  // quantities (force) instead of 6 (force, torque)
  constexpr bool COM = SL == 1 && SC + SD + SQ == 0 && !MIX;
  constexpr int NT = COM ? 3 : 6;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  unsigned char *list = lists[wave];
  int *scnt = scnts[wave];
  const int cell = xcd_remap(blockIdx.x, gridDim.x);
  const bool full = o.nq > 6;
  const int nwords = NT + (full ? 4 : 0);
  int *const jhi = (int *)(jacc + nwords * CAP);
  R *const rft = (R *)o.rows;
  const double shift0 = md->shift_sum[0][0];
  const LJPair lj0 = md->lj[0][0][0][0];
  double acc5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (cell < c.ncell) {
    const int hs = c.cell_start[cell];
    const int hn = __builtin_amdgcn_readfirstlane(c.cell_start[cell + 1] - hs);
    if (tid < 64) build_nb<true>(c, cell, nb);
    __syncthreads();
    const int M = nb.off[14];
    if (hn == 0) {  // no home molecules: the partner rows of the half neighbourhood are zero
      for (int g = tid; g < M; g += 64 * W) {
        const int k = find_nb(nb.off, g);
        const int64_t ent = (int64_t)(1 + k) * o.n + nb.start[k] + (g - nb.off[k]);
        for (int q = 0; q < NT; ++q) rft[NT * ent + q] = (R)0;
        if (full)
          for (int q = 0; q < 3; ++q) o.rows_uw[3 * ent + q] = 0.0;
      }
    }
    for (int ic = 0; ic < hn; ic += 64 * W) {
      // this round's molecules, split evenly over the wavefronts (wave-uniform)
      const int rem = min(64 * W, hn - ic), base = rem / W, extra = rem % W;
      const int hc = base + (wave < extra ? 1 : 0);
      const int i0 = ic + wave * base + min(wave, extra);
      const float rhc = __builtin_amdgcn_rcpf((float)(hc > 0 ? hc : 1));
      const int NS = hc > 0 ? min(8, div_small(64, rhc)) : 1;
      const int sl = hc > 0 ? div_small(lane, rhc) : NS, il = hc > 0 ? lane - sl * hc : 0;
      const float rns = __builtin_amdgcn_rcpf((float)NS);
      const bool act = sl < NS;
      const int sla = act ? sl : 0;
      const int iloc = i0 + il;
      double xi = 1e30, yi = 1e30, zi = 1e30;  // idle lanes: no candidate is within the cutoff
      R vi[NV][3];
      double vil[SL][3];
      int ci = 0;
      {
        const int sidx = hs + (hc > 0 ? iloc : 0);
        if (act) xi = c.sx[sidx], yi = c.sy[sidx], zi = c.sz[sidx];
        if (MIX) ci = c.scomp[sidx];
        if constexpr (!COM) {
          const double *v = c.svec + (int64_t)sidx * NV * 3;
#pragma unroll
          for (int k = 0; k < NV; ++k) vi[k][0] = (R)v[3 * k], vi[k][1] = (R)v[3 * k + 1], vi[k][2] = (R)v[3 * k + 2];
#pragma unroll
          for (int k = 0; k < SL; ++k) vil[k][0] = v[3 * k], vil[k][1] = v[3 * k + 1], vil[k][2] = v[3 * k + 2];
        }
      }
      double fx = 0.0, fy = 0.0, fz = 0.0, tx = 0.0, ty = 0.0, tz = 0.0, uu = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
      double ush = 0.0;  // LJTS shifts of the interacting molecule pairs (mixtures)
      int nn = 0;
      int cnt = 0;
      unsigned char *mylist = list + lane;
      // pass 2 over the listed hits of the current window
      auto flush = [&]() {
        scnt[lane] = cnt;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (act) {
          unsigned H = 0;
#pragma unroll
          for (int s2 = 0; s2 < 8; ++s2)
            if (s2 < NS) H += (unsigned)scnt[il + s2 * hc];
          const unsigned q0 = (unsigned)div_small((int)H * sl, rns), q1 = (unsigned)div_small((int)H * (sl + 1), rns);
          // locate hit q0 (list sp, entry j); each iteration loads the next entry ahead
          unsigned j = q0, csp = (unsigned)scnt[il];
          int sp = 0;
          if (q0 < q1)
            while (j >= csp) j -= csp, ++sp, csp = (unsigned)scnt[il + sp * hc];
          int li = il + sp * hc + 64 * (int)j;
          int un = q0 < q1 ? list[li] : 0;
          for (unsigned q = q0; q < q1; ++q) {
            const int u = un;
            if (q + 1 < q1) {
              ++j, li += 64;
              while (j >= csp) j = 0, ++sp, csp = (unsigned)scnt[il + sp * hc], li = il + sp * hc;
              un = list[li];
            }
            const double dx = xi - jp[3 * u], dy = yi - jp[3 * u + 1], dz = zi - jp[3 * u + 2];
            const int cj = MIX ? jc_[u] : 0;
            double F0, F1, F2, T0 = 0.0, T1 = 0.0, T2 = 0.0, up;
            if constexpr (COM) {
              // LJ between the centres: the separation is the COM separation, in FP64 throughout
              const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
              const double ir2d = rcp_fp64_from<R>(r2);
              const double s2d = lj0.sig2 * ir2d;
              const double s6d = s2d * s2d * s2d;
              up = (lj0.eps4 * s6d) * (s6d - 1.0);
              const double fs = (lj0.eps24 * ir2d) * (s6d * fma(2.0, s6d, -1.0));
              F0 = fs * dx, F1 = fs * dy, F2 = fs * dz;
              fx += F0, fy += F1, fz += F2;
            } else {
              PairAcc<R> acc{{0, 0, 0}, {0, 0, 0}, 0};
              mol_pair<SL, SC, SD, SQ, MIX, R>(md, ci, cj, vil, vi, jl[u], jv[u], dx, dy, dz, acc);
              addto(fx, acc.F[0]), addto(fy, acc.F[1]), addto(fz, acc.F[2]);
              addto(tx, acc.T[0]), addto(ty, acc.T[1]), addto(tz, acc.T[2]);
              F0 = acc.F[0], F1 = acc.F[1], F2 = acc.F[2];
              T0 = -(double)acc.T[0] - fma(dy, F2, -(dz * F1));  // partner: -tau - d x F
              T1 = -(double)acc.T[1] - fma(dz, F0, -(dx * F2));
              T2 = -(double)acc.T[2] - fma(dx, F1, -(dy * F0));
              up = acc.u;
            }
            uu += up;
            const double dw = fma(dz, F2, fma(dy, F1, dx * F0));
            wx = fma(dx, F0, wx);
            wy = fma(dy, F1, wy);
            wz = fma(dz, F2, wz);
            const double sh = MIX ? md->shift_sum[ci][cj] : shift0;
            if (MIX) ush += sh;
            nn += 1;
            const double pv[6] = {-F0, -F1, -F2, T0, T1, T2};  // the partner's force and torque
            bool ok = true;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
              if constexpr (F64) ok &= fx2_add(&jacc[q * CAP + u], &jhi[q * CAP + u], pv[q]);
              else ok &= fx1_add(&jacc[q * CAP + u], pv[q]);
            }
            if (full) {
              ok &= fx_add(&jacc[NT * CAP + u], &jacc[(NT + 1) * CAP + u], 0.5 * (up - sh));
              ok &= fx_add(&jacc[(NT + 2) * CAP + u], &jacc[(NT + 3) * CAP + u], 0.5 * dw);
            }
            if (!ok) jbad[u] = 1;
            atomicAdd(&jn[u], 1u);
          }
        }
        cnt = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      };
      for (int jc = 0; jc < M; jc += CAP) {
        const int mj = min(CAP, M - jc);
        __syncthreads();
        for (int t = tid; t < mj; t += 64 * W) {
          const int g = jc + t;
          const int k = find_nb(nb.off, g);
          const int src = nb.start[k] + (g - nb.off[k]);
          jp[3 * t] = c.sx[src] + nb.sh[k][0];
          jp[3 * t + 1] = c.sy[src] + nb.sh[k][1];
          jp[3 * t + 2] = c.sz[src] + nb.sh[k][2];
          if (MIX) jc_[t] = c.scomp[src];  // written (clamped to [0, ncomp)) by the gather
          if constexpr (!COM) {
            const double *v = c.svec + (int64_t)src * NV * 3;
#pragma unroll
            for (int q = 0; q < SL * 3; ++q) jl[t][q] = v[q];
#pragma unroll
            for (int q = SL * 3; q < NV * 3; ++q) jv[t][q - SL * 3] = (R)v[q];
          }
          for (int q = 0; q < nwords; ++q) jacc[q * CAP + t] = 0ull;
          if constexpr (F64)
            for (int q = 0; q < NT; ++q) jhi[q * CAP + t] = 0;
          jn[t] = 0u;
          jbad[t] = 0;
        }
        __syncthreads();
        if (hc > 0) {
          const int self = iloc - jc;  // window slot of the molecule itself (may be outside)
          int kb = 0;
          while (true) {
            // pass 1: walk until the window ends or a list could overflow; the slot is always
            // written, the count advances on a hit
            for (; kb < mj && !__any(cnt > LCAP - 2); kb += 2 * NS) {
              const int ta = kb + sla, tb = ta + NS;
              const double ax = xi - jp[3 * ta], ay = yi - jp[3 * ta + 1], az = zi - jp[3 * ta + 2];
              const double bx_ = xi - jp[3 * tb], by_ = yi - jp[3 * tb + 1], bz_ = zi - jp[3 * tb + 2];
              const double ra = fma(az, az, fma(ay, ay, ax * ax));
              const double rb = fma(bz_, bz_, fma(by_, by_, bx_ * bx_));
              mylist[64 * cnt] = (unsigned char)ta;
              cnt += (ta < mj && ra < rc2 && ta > self) ? 1 : 0;
              mylist[64 * cnt] = (unsigned char)tb;
              cnt += (tb < mj && rb < rc2 && tb > self) ? 1 : 0;
            }
            flush();
            if (kb >= mj) break;
          }
        }
        __syncthreads();
        // partner sums of this window to the rows (later rounds add to the first round's)
        for (int t = tid; t < mj; t += 64 * W) {
          const int g = jc + t;
          const int k = find_nb(nb.off, g);
          const int64_t ent = (int64_t)(1 + k) * o.n + nb.start[k] + (g - nb.off[k]);
          const unsigned K = jn[t];
          const bool bad = jbad[t] != 0;
          if (bad) {  // NaN here; listed for the FP64 fix-up
            const unsigned long long e = atomicAdd(o.bad, 1ull);
            if (e < BAD_CAP) o.bad[1 + e] = (unsigned long long)ent;
            else atomicOr(o.status, MD_DEV_RANGE);
          }
#pragma unroll 1
          for (int q = 0; q < NT + (full ? 3 : 0); ++q) {
            const int w = q < NT ? q : NT + 2 * (q - NT);  // first word of quantity q
            const double v = q == NT + 2 ? (double)K
                             : bad       ? __builtin_nan("")
                             : q >= NT   ? fx_value(jacc[w * CAP + t], jacc[(w + 1) * CAP + t], K)
                             : F64       ? fx2_value(jacc[w * CAP + t], jhi[(q < NT ? q : 0) * CAP + t], K)
                                         : fx1_value(jacc[w * CAP + t], K);
            if (q < NT) rft[NT * ent + q] = ic == 0 ? (R)v : (R)((double)rft[NT * ent + q] + v);
            else o.rows_uw[3 * ent + q - NT] = ic == 0 ? v : o.rows_uw[3 * ent + q - NT] + v;
          }
        }
      }
      uu -= MIX ? ush : (double)nn * shift0;
      // slices of molecule il sit in lanes il + s hc: add them to lane il in slice order
      double dn = (double)nn;
      for (int s2 = 1; s2 < NS; ++s2) {
        const int src = lane + s2 * hc;  // meaningful for lane < hc
        const double f0 = __shfl(fx, src), f1 = __shfl(fy, src), f2 = __shfl(fz, src);
        const double t0 = __shfl(tx, src), t1 = __shfl(ty, src), t2 = __shfl(tz, src);
        const double u0 = __shfl(uu, src), w0 = __shfl(wx, src), w1 = __shfl(wy, src), w2 = __shfl(wz, src);
        const double n0 = __shfl(dn, src);
        if (lane < hc)
          fx += f0, fy += f1, fz += f2, tx += t0, ty += t1, tz += t2, uu += u0, wx += w0, wy += w1, wz += w2,
              dn += n0;
      }
      if (lane < hc) {
        R *row = rft + NT * (int64_t)(hs + iloc);  // row 0: the molecule's own sums
        row[0] = (R)fx, row[1] = (R)fy, row[2] = (R)fz;
        if constexpr (!COM) row[3] = (R)tx, row[4] = (R)ty, row[5] = (R)tz;
        if (full) {
          double *ru = o.rows_uw + 3 * (int64_t)(hs + iloc);
          ru[0] = 0.5 * uu, ru[1] = 0.5 * (wx + wy + wz), ru[2] = dn;
        }
        // each pair once: U, W and W_aa in full, the partner count twice (the sum of nnb_mol)
        acc5[0] += uu, acc5[1] += wx, acc5[2] += wy, acc5[3] += wz, acc5[4] += 2.0 * dn;
      }
    }
  }
  write_partial_block<W>(o.partial, acc5, red);
}

// Partner rows listed by the pair kernel because a term left the range of the exact LDS sums
// (overlapping molecules): each such row is formed again from scratch, every term evaluated as
// pass 2 evaluates it (same cutoff arithmetic, same pair function, partner terms by the same
// identities) and summed in FP64.  One wavefront per row: lane l takes the home molecules
// l, l + 64, ... in turn, and each round of 64 terms is added by a fixed butterfly, read from
// lane 0, so the sum is the same on every run.
template <typename R, int SL, int SC, int SD, int SQ, bool MIX>
__global__ __launch_bounds__(64) void k_pair_fixup(CellsDev c, const ModelDev *__restrict__ md, double rc2,
                                                   PairOut o) {
  constexpr int NV = Slots<SL, SC, SD, SQ>::nv;
  constexpr int NE = NV - SL > 0 ? NV - SL : 1;
  constexpr bool COM = SL == 1 && SC + SD + SQ == 0 && !MIX;
  constexpr int NT = COM ? 3 : 6;
  const unsigned long long cnt = min(o.bad[0], (unsigned long long)BAD_CAP);
  const bool full = o.nq > 6;
  const int lane = threadIdx.x;
  for (unsigned long long e = blockIdx.x; e < cnt; e += gridDim.x) {
    const int64_t ent = (int64_t)o.bad[1 + e];
    const int k = (int)(ent / o.n) - 1;  // half-stencil entry of the partner's cell
    const int64_t src = ent - (int64_t)(k + 1) * o.n;
    // the partner's cell B: cell_start[B] <= src < cell_start[B + 1]
    int lo = 0, hi = c.ncell;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (c.cell_start[mid] <= src) lo = mid;
      else hi = mid;
    }
    const int B = lo;
    // home cell A = B - offset (wrapped) and the image shift of B seen from A, as build_nb forms it
    const int e13 = k + 13, ox = e13 % 3 - 1, oy = (e13 / 3) % 3 - 1, oz = e13 / 9 - 1;
    int ax = B % c.nx - ox, ay = (B / c.nx) % c.ny - oy, az = B / (c.nx * c.ny) - oz;
    ax += ax < 0 ? c.nx : (ax >= c.nx ? -c.nx : 0);
    ay += ay < 0 ? c.ny : (ay >= c.ny ? -c.ny : 0);
    az += az < 0 ? c.nz : (az >= c.nz ? -c.nz : 0);
    const double shx = ax + ox < 0 ? -c.Lx : (ax + ox >= c.nx ? c.Lx : 0.0);
    const double shy = ay + oy < 0 ? -c.Ly : (ay + oy >= c.ny ? c.Ly : 0.0);
    const double shz = az + oz < 0 ? -c.Lz : (az + oz >= c.nz ? c.Lz : 0.0);
    const int A = (az * c.ny + ay) * c.nx + ax;
    const double jx = c.sx[src] + shx, jy = c.sy[src] + shy, jz = c.sz[src] + shz;
    double jl[SL * 3];
    R jv[NE * 3];
    if constexpr (!COM) {
      const double *v = c.svec + src * NV * 3;
#pragma unroll
      for (int q = 0; q < SL * 3; ++q) jl[q] = v[q];
#pragma unroll
      for (int q = SL * 3; q < NV * 3; ++q) jv[q - SL * 3] = (R)v[q];
    }
    const int cj = MIX ? c.scomp[src] : 0;
    const int as = c.cell_start[A], an = c.cell_start[A + 1] - as;
    double sum[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < an; i0 += 64) {
      const int i = i0 + lane;
      double v[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      // own cell: partners after the molecule only
      if (i < an && !(k == 0 && src - as <= i)) {
        const int sidx = as + i;
        const double dx = c.sx[sidx] - jx, dy = c.sy[sidx] - jy, dz = c.sz[sidx] - jz;
        if (COM && fma(dz, dz, fma(dy, dy, dx * dx)) < rc2) {
          const LJPair &p = md->lj[0][0][0][0];
          const double ir2d = rcp_fp64_from<R>(fma(dz, dz, fma(dy, dy, dx * dx)));
          const double s2d = p.sig2 * ir2d;
          const double s6d = s2d * s2d * s2d;
          const double fs = (p.eps24 * ir2d) * (s6d * fma(2.0, s6d, -1.0));
          const double F0 = fs * dx, F1 = fs * dy, F2 = fs * dz;
          v[0] = -F0, v[1] = -F1, v[2] = -F2;
          v[6] = 0.5 * ((p.eps4 * s6d) * (s6d - 1.0) - md->shift_sum[0][0]);
          v[7] = 0.5 * fma(dz, F2, fma(dy, F1, dx * F0));
          v[8] = 1.0;
        } else if (!COM && fma(dz, dz, fma(dy, dy, dx * dx)) < rc2) {
          R vi[NV][3];
          double vil[SL][3];
          const double *w = c.svec + (int64_t)sidx * NV * 3;
#pragma unroll
          for (int q = 0; q < NV; ++q) vi[q][0] = (R)w[3 * q], vi[q][1] = (R)w[3 * q + 1], vi[q][2] = (R)w[3 * q + 2];
#pragma unroll
          for (int q = 0; q < SL; ++q) vil[q][0] = w[3 * q], vil[q][1] = w[3 * q + 1], vil[q][2] = w[3 * q + 2];
          const int ci = MIX ? c.scomp[sidx] : 0;
          PairAcc<R> acc{{0, 0, 0}, {0, 0, 0}, 0};
          mol_pair<SL, SC, SD, SQ, MIX, R>(md, ci, cj, vil, vi, jl, jv, dx, dy, dz, acc);
          const double F0 = acc.F[0], F1 = acc.F[1], F2 = acc.F[2];
          v[0] = -F0, v[1] = -F1, v[2] = -F2;
          v[3] = -(double)acc.T[0] - fma(dy, F2, -(dz * F1));
          v[4] = -(double)acc.T[1] - fma(dz, F0, -(dx * F2));
          v[5] = -(double)acc.T[2] - fma(dx, F1, -(dy * F0));
          v[6] = 0.5 * (acc.u - md->shift_sum[ci][cj]);
          v[7] = 0.5 * fma(dz, F2, fma(dy, F1, dx * F0));
          v[8] = 1.0;
        }
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v[q] += __shfl_xor(v[q], m);
        sum[q] += v[q];
      }
    }
    if (lane == 0) {
      R *row = (R *)o.rows + NT * ent;
      for (int q = 0; q < NT; ++q) row[q] = (R)sum[q];
      if (full) o.rows_uw[3 * ent] = sum[6], o.rows_uw[3 * ent + 1] = sum[7], o.rows_uw[3 * ent + 2] = sum[8];
    }
  }
}

// Sum of the N3_ROWS rows of every molecule and quantity in row order (in FP64), written in the
// caller's molecule order (thread per molecule and quantity; row reads coalesced).
template <typename R, int NT, int NQ>
__global__ __launch_bounds__(256) void k_pair_gather(const int32_t *__restrict__ perm, PairOut o) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) o.bad[0] = 0ull;  // the fix-up has run
  if (t >= o.n * NQ) return;
  const int64_t s = t / NQ;
  const int q = (int)(t - s * NQ);
  double v;
  if (q < NT) {
    const R *rows = (const R *)o.rows + NT * s + q;
    v = (double)rows[0];
#pragma unroll
    for (int r = 1; r < N3_ROWS; ++r) v += (double)rows[r * NT * o.n];
  } else {
    const double *rows = o.rows_uw + 3 * s + q - NT;
    v = rows[0];
#pragma unroll
    for (int r = 1; r < N3_ROWS; ++r) v += rows[r * 3 * o.n];
  }
  const int64_t orig = perm[s];
  if (q < 3) {
    o.force[3 * orig + q] = v;
    if (NT == 3 && o.torque) o.torque[3 * orig + q] = 0.0;  // a centre-only site has no torque
  } else if (q < NT) {
    if (o.torque) o.torque[3 * orig + q - 3] = v;
  } else if (q == NT) {
    if (o.u_mol) o.u_mol[orig] = v;
  } else if (q == NT + 1) {
    if (o.w_mol) o.w_mol[orig] = v;
  } else if (o.nnb_mol) {
    o.nnb_mol[orig] = (int32_t)v;
  }
}

// ---------------------------------------------------------------- deterministic reductions
constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 256;
constexpr int RED_MAXCOLS = 256;

// Column sums of a [nrows][ncols] table (optionally followed by the columns of a second table
// [nrows2][ncols2]) in two launches.  Stage 1: block b sums rows [b chunk, (b + 1) chunk), thread
// t taking rows t, t + 256, ... in order, then a fixed LDS tree, into red2[b]; the same for the
// second table with its own chunk.  Stage 2 (one block) sums red2 over b in the same way and writes
// the result, for the force sums also U, W, W_aa, the pair count and the energies row (with the
// kinetic energies of the leapfrog as the second table).  The summation order never depends on
// timing.
__device__ __forceinline__ double block_tree(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_cols(const double *rows, int64_t nrows, int ncols,
                                                             int64_t chunk, const double *rows2, int64_t nrows2,
                                                             int ncols2, int64_t chunk2, double *out) {
  __shared__ double sh[RED_THREADS];
  const int nc = ncols + ncols2;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(nrows, r0 + chunk);
  for (int col = 0; col < ncols; ++col) {
    double v = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += RED_THREADS) v += rows[r * ncols + col];
    v = block_tree(v, sh);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * nc + col] = v;
  }
  const int64_t q0 = (int64_t)blockIdx.x * chunk2;
  const int64_t q1 = min(nrows2, q0 + chunk2);
  for (int col = 0; col < ncols2; ++col) {
    double v = 0.0;
    for (int64_t r = q0 + threadIdx.x; r < q1; r += RED_THREADS) v += rows2[r * ncols2 + col];
    v = block_tree(v, sh);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * nc + ncols + col] = v;
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(const double *red2, int nb, int ncols, double *out,
                                                              int finish, double *uw, int64_t *npairs, double *erow) {
  __shared__ double sh[RED_THREADS];
  __shared__ double res[RED_MAXCOLS];
  for (int col = 0; col < ncols; ++col) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += RED_THREADS) v += red2[(int64_t)b * ncols + col];
    v = block_tree(v, sh);
    if (threadIdx.x == 0) res[col] = v;
  }
  if (threadIdx.x != 0) return;
  if (finish) {
    const double U = res[0], W = res[1] + res[2] + res[3];
    uw[0] = U, uw[1] = W, uw[2] = res[1], uw[3] = res[2], uw[4] = res[3];
    if (npairs) *npairs = (int64_t)(res[4] * 0.5);
    if (erow) erow[0] = U, erow[3] = W;
    if (ncols == PARTIAL_COLS + KIN_COLS) {
      if (erow) erow[1] = res[PARTIAL_COLS], erow[2] = res[PARTIAL_COLS + 1];
      uw[5] = res[PARTIAL_COLS], uw[6] = res[PARTIAL_COLS + 1], uw[7] = res[PARTIAL_COLS + 2];
    }
  } else {
    for (int col = 0; col < ncols; ++col) out[col] = res[col];
  }
}

// Dense cells (mean occupancy >= 16) are shared by four wavefronts and staged in larger windows;
// sparser ones take one wavefront each.  The partner sums take 8 bytes per word and slot of
// dynamic LDS.  Window sizes and waves per SIMD are chosen per shape and precision so that the
// LDS of three blocks (or of two where the registers allow only two waves) fits a CU.  The
// gather then forms every molecule's results from its rows.
template <typename R, int SL, int SC, int SD, int SQ, bool MIX, int CAP1, int CAP4, int WPE>
int launch_ms(const CellsDev &cd, const md_model *m, const PairOut &o, int64_t nb, double mean, hipStream_t s) {
  constexpr int NT = SL == 1 && SC + SD + SQ == 0 && !MIX ? 3 : 6;  // partner force (and torque) quantities
  const bool full = o.nq > 6;
  const size_t per_slot = (size_t)(NT + (full ? 4 : 0)) * sizeof(unsigned long long) + (sizeof(R) == 8 ? NT * sizeof(int) : 0);
  if (mean >= 16.0)
    k_pair_ms<R, SL, SC, SD, SQ, MIX, CAP4, 4, WPE>
        <<<(unsigned)nb, 256, per_slot * CAP4, s>>>(cd, m->dev, m->host.rc2, o);
  else
    k_pair_ms<R, SL, SC, SD, SQ, MIX, CAP1, 1, WPE>
        <<<(unsigned)nb, 64, per_slot * CAP1, s>>>(cd, m->dev, m->host.rc2, o);
  int rc = check_hip(hipGetLastError(), "k_pair_ms");
  if (rc || o.n == 0) return rc;
  k_pair_fixup<R, SL, SC, SD, SQ, MIX><<<256, 64, 0, s>>>(cd, m->dev, m->host.rc2, o);
  if ((rc = check_hip(hipGetLastError(), "k_pair_fixup"))) return rc;
  const unsigned gb = (unsigned)((o.n * (NT + (full ? 3 : 0)) + 255) / 256);
  if (full) k_pair_gather<R, NT, NT + 3><<<gb, 256, 0, s>>>(cd.perm, o);
  else k_pair_gather<R, NT, NT><<<gb, 256, 0, s>>>(cd.perm, o);
  return check_hip(hipGetLastError(), "k_pair_gather");
}

}  // namespace

// Scratch of md_forces_noalloc: one array per GPU, for the life of the process.  In host code
// `scratch` names a host-side stand-in, never the device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) static unsigned char scratch[MD_NOALLOC_SCRATCH_BYTES];

int noalloc_scratch(void **ptr) {
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static void *addr[MAXDEV] = {};
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= MAXDEV) return set_error(MD_EINVAL, "md_forces_noalloc: device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    if ((rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return rc;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return MD_OK;
}

CellsDev cells_dev(const md_cells *c) {
  CellsDev d;
  d.cell_start = c->sub ? c->cstart : c->start;
  d.sub_start = c->sub ? c->start : nullptr;
  d.perm = c->perm;
  d.scomp = c->scomp;
  d.sx = c->sx, d.sy = c->sy, d.sz = c->sz;
  d.svec = c->svec;
  d.squat = c->squat;
  d.nx = c->nc[0], d.ny = c->nc[1], d.nz = c->nc[2];
  d.ncell = (int32_t)c->ncell;
  d.nvec = c->nvec;
  d.Lx = c->box[0], d.Ly = c->box[1], d.Lz = c->box[2];
  d.hx = c->box[0] / c->nc[0], d.hy = c->box[1] / c->nc[1], d.hz = c->box[2] / c->nc[2];
  return d;
}

int launch_pair(md_model *m, const md_cells *c, int precision, const PairOut &o, hipStream_t s, int64_t *nblocks) {
  const CellsDev cd = cells_dev(c);
  const int64_t nb = pair_blocks(c->ncell);
  *nblocks = nb;
  const bool f32 = precision == MD_FP32;
  if (m->single_site && (m->flags & MD_HALF_SHELL)) {  // the half-shell kernel, centre-only shape
    const double mean = (double)c->N / (double)c->ncell;
    return f32 ? launch_ms<float, 1, 0, 0, 0, false, 96, 256, 3>(cd, m, o, nb, mean, s)
               : launch_ms<double, 1, 0, 0, 0, false, 96, 256, 3>(cd, m, o, nb, mean, s);
  }
  if (m->single_site) {
    const LJPair &p = m->host.lj[0][0][0][0];
    const LJK k{p.eps4, p.eps24, p.sig2, p.shift, m->host.rc2, (float)p.eps24, (float)p.sig2,
                lj_guard_threshold(m->host.rc, cd.hx, cd.hy, cd.hz)};
    int cap = lj1_tile_cap(c->N, c->ncell);
    int lcap = lj1_list_cap(c->N, c->box[0] * c->box[1] * c->box[2], m->host.rc, c->ncell);
    // tile (FP32 copy on the FP32 path, FP64 positions; at least the 16 KiB of the slice sums),
    // then per-lane and per-molecule hit lists
    auto dyn_lds = [f32](int cp, int lc) {
      return std::max((size_t)cp * (f32 ? 40 : 24), (size_t)256 * 8 * sizeof(double)) +
             (size_t)lc * 256 * sizeof(unsigned short);
    };
    // stay within the device's LDS per block: shrink the tile first (tiles beyond it take the
    // windowed walk), then the hit lists (which flush earlier); results do not depend on either
    // beyond rounding
    if (!m->lds_limit) {
      int dev = 0, v = 0;
      if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        m->lds_limit = v;
      else
        m->lds_limit = 64 * 1024;
    }
    const bool sub = c->sub;
    // the static LDS of the instances (the same for both WPE variants)
    const void *kf = sub ? (f32 ? (const void *)k_pair_lj<float, true, 4> : (const void *)k_pair_lj<double, true, 4>)
                         : (f32 ? (const void *)k_pair_lj<float, false, 4> : (const void *)k_pair_lj<double, false, 4>);
    const int kv = (int)f32 + 2 * (int)sub;
    if (m->lj1_static_lds[kv] < 0) {
      hipFuncAttributes fa{};
      m->lj1_static_lds[kv] = hipFuncGetAttributes(&fa, kf) == hipSuccess ? (int)fa.sharedSizeBytes : 4096;
    }
    const size_t stat = (size_t)m->lj1_static_lds[kv];
    while (stat + dyn_lds(cap, lcap) > (size_t)m->lds_limit && cap > 256) cap = std::max(256, cap - 64);
    while (stat + dyn_lds(cap, lcap) > (size_t)m->lds_limit && lcap > 16) lcap -= 4;
    const size_t lds = dyn_lds(cap, lcap);
    const int64_t nq = pair_blocks((int64_t)c->nc[0] * ((c->nc[1] + 1) / 2) * ((c->nc[2] + 1) / 2));
    *nblocks = nq;
    // blocks per CU that the LDS allows decides the register budget of the instance
    if (!m->lds_per_cu) {
      int dev = 0, v = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess && v > 0)
        m->lds_per_cu = v;
      else
        m->lds_per_cu = 160 * 1024;
    }
    const bool w5 = (size_t)m->lds_per_cu / (stat + lds) >= 5;
#define MD_LJ_LAUNCH(RR, SS)                                                                 \
  (w5 ? k_pair_lj<RR, SS, 5><<<(unsigned)nq, 256, lds, s>>>(cd, k, o, cap, lcap)             \
      : k_pair_lj<RR, SS, 4><<<(unsigned)nq, 256, lds, s>>>(cd, k, o, cap, lcap))
    if (sub && f32) MD_LJ_LAUNCH(float, true);
    else if (sub) MD_LJ_LAUNCH(double, true);
    else if (f32) MD_LJ_LAUNCH(float, false);
    else MD_LJ_LAUNCH(double, false);
#undef MD_LJ_LAUNCH
    return check_hip(hipGetLastError(), "k_pair_lj");
  }
  const Shape &S = m->shape;
  const double mean = (double)c->N / (double)c->ncell;
  if (m->fixed_shape && S.lj == 2 && S.chg == 0 && S.dip == 0 && S.quad == 1)
    return f32 ? launch_ms<float, 2, 0, 0, 1, false, 64, 256, 3>(cd, m, o, nb, mean, s)
               : launch_ms<double, 2, 0, 0, 1, false, 64, 192, 3>(cd, m, o, nb, mean, s);
  if (m->fixed_shape && S.lj == 3 && S.chg == 0 && S.dip == 1 && S.quad == 0)
    return f32 ? launch_ms<float, 3, 0, 1, 0, false, 64, 224, 3>(cd, m, o, nb, mean, s)
               : launch_ms<double, 3, 0, 1, 0, false, 64, 192, 3>(cd, m, o, nb, mean, s);
  return f32 ? launch_ms<float, MD_MAX_LJ, MD_MAX_CHG, MD_MAX_DIP, MD_MAX_QUAD, true, 64, 128, 1>(cd, m, o, nb, mean, s)
             : launch_ms<double, MD_MAX_LJ, MD_MAX_CHG, MD_MAX_DIP, MD_MAX_QUAD, true, 64, 96, 1>(cd, m, o, nb, mean, s);
}

int launch_reduce(md_model *m, int64_t nrows, int ncols, const double *rows, double *out, hipStream_t s) {
  if (ncols > RED_MAXCOLS) return set_error(MD_EINVAL, "reduction too wide");
  const int64_t chunk = (nrows + RED_BLOCKS - 1) / RED_BLOCKS;
  k_reduce_cols<<<RED_BLOCKS, RED_THREADS, 0, s>>>(rows, nrows, ncols, chunk > 0 ? chunk : 1, nullptr, 0, 0, 1,
                                                   m->red2);
  k_reduce_final<<<1, RED_THREADS, 0, s>>>(m->red2, RED_BLOCKS, ncols, out, 0, nullptr, nullptr, nullptr);
  return check_hip(hipGetLastError(), "k_reduce");
}

int launch_reduce_forces(md_model *m, int64_t nrows, const double *rows, double *uw, int64_t *npairs, double *erow,
                         hipStream_t s, const double *kin_rows, int64_t kin_nrows) {
  const int64_t chunk = (nrows + RED_BLOCKS - 1) / RED_BLOCKS;
  const int kc = kin_rows ? KIN_COLS : 0;
  const int64_t chunk2 = (kin_nrows + RED_BLOCKS - 1) / RED_BLOCKS;
  k_reduce_cols<<<RED_BLOCKS, RED_THREADS, 0, s>>>(rows, nrows, PARTIAL_COLS, chunk > 0 ? chunk : 1, kin_rows,
                                                   kc ? kin_nrows : 0, kc, chunk2 > 0 ? chunk2 : 1, m->red2);
  k_reduce_final<<<1, RED_THREADS, 0, s>>>(m->red2, RED_BLOCKS, PARTIAL_COLS + kc, nullptr, 1, uw, npairs, erow);
  return check_hip(hipGetLastError(), "k_reduce");
}

}  // namespace mdcell
