// Linked-cell build: periodic wrap, cell assignment, stable counting sort into cells, and the
// sorted structure-of-arrays gather with the world-frame site transform (Sec. 3, linked-cell
// paragraphs; periodic boundaries; rigid molecules oriented by quaternions, Sec. 3 Eqs. 4-5).
//
// HBM-bound: per molecule the build reads the COM (24 B), id/slot words and, for multi-site
// models, the quaternion (32 B) and component id, and writes cell id, slot, permutation and the
// sorted COM copy (24 B) plus site vectors.  Launch shapes are 256-thread blocks over molecules.
// Five launches: bin (+ histogram), tile scan, scan of tile totals, scatter (+ final cell
// starts), rank + gather.  The scan leaves the histogram zeroed for the next build.

#include <algorithm>

#include "md_internal.h"

namespace mdcell {
namespace {

__device__ __forceinline__ int bin1(double xw, double inv_h, int n) {
  int c = (int)floor(xw * inv_h);
  return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
}

struct BinArgs {
  const double *pos, *quat;
  const int32_t *comp, *order;  // order: visiting order (the previous build's permutation) or NULL
  int64_t N;
  double Lx, Ly, Lz, ihx, ihy, ihz;
  double ihx2, ihy2, ihz2;  // 2 n_k / L_k: half-edge cells (sub)
  int32_t nx, ny, nz, ncomp, check_quat, sub;
  int32_t *cellv, *slotv, *count, *status;
};

// Low bit of the half-edge cell index min(2 n - 1, floor(xw * (2 n / L))) along one axis: which
// half of its cell the coordinate lies in.
__device__ __forceinline__ int half_bit(double xw, double inv_hh, int n) { return bin1(xw, inv_hh, 2 * n) & 1; }

// Wrap + bin + per-bin histogram (a bin is a cell, or with half-edge cells the half-cell 8 cell +
// octant, octant 4 z + 2 y + x from the low bits of the half-cell coordinates).  Position d of
// the visiting order takes molecule order[d] (identity without an order) and writes its bin and
// provisional slot at position d (coalesced).
// In the previous build's order neighbouring positions mostly fall into the same cell, and each
// run of equal cells inside a wavefront takes one atomic add.  The blocks of each XCD (block b
// runs on XCD b % 8) take one contiguous eighth of the positions, so the COM lines a region of
// space gathers meet in one L2.  The final order inside a cell is fixed by k_rank_gather.
__global__ __launch_bounds__(256) void k_bin(BinArgs a) {
  const int64_t d = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = d < a.N;
  const int64_t i = valid ? (a.order ? (int64_t)a.order[d] : d) : 0;
  double x = a.pos[3 * i], y = a.pos[3 * i + 1], z = a.pos[3 * i + 2];
  int flags = 0;
  const bool finite = isfinite(x) && isfinite(y) && isfinite(z);
  if (!finite) {
    flags |= MD_DEV_NONFINITE;
    x = y = z = 0.0;
  }
  if (a.comp) {
    const int32_t c = a.comp[i];
    if (c < 0 || c >= a.ncomp) flags |= MD_DEV_COMP;
  }
  if (a.check_quat && a.quat) {
    const double *q = a.quat + 4 * i;
    const double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(fabs(n2 - 1.0) <= 1e-6)) flags |= MD_DEV_QUAT;
  }
  if (flags && valid) atomicOr(a.status, flags);
  const double xw = wrap1(x, a.Lx), yw = wrap1(y, a.Ly), zw = wrap1(z, a.Lz);
  const int cx = bin1(xw, a.ihx, a.nx);
  const int cy = bin1(yw, a.ihy, a.ny);
  const int cz = bin1(zw, a.ihz, a.nz);
  // a molecule with a non-finite coordinate goes to cell i mod ncell, so that such molecules
  // (a run that blew up) spread over the grid instead of crowding one cell; its sorted copy is
  // NaN, which fails every cutoff test, so it has no partners
  int cell = !valid ? -1 : (finite ? (cz * a.ny + cy) * a.nx + cx : (int)(i % (int64_t)(a.nx * a.ny * a.nz)));
  if (a.sub && valid)
    cell = 8 * cell + (finite ? 4 * half_bit(zw, a.ihz2, a.nz) + 2 * half_bit(yw, a.ihy2, a.ny) + half_bit(xw, a.ihx2, a.nx)
                              : 0);
  // runs of equal cells among consecutive lanes: the run head adds the run length
  const int prev = __shfl_up(cell, 1, 64);
  const bool head = lane == 0 || prev != cell;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1);
  const int hl = 63 - __clzll(heads & upto);  // this lane's run head
  const unsigned long long after = heads & ~upto;
  const int next = after ? __ffsll(after) - 1 : 64;  // first head after this lane
  int base = 0;
  if (head && valid) base = atomicAdd(a.count + cell, next - lane);
  base = __shfl(base, hl, 64);
  if (valid) {
    a.cellv[d] = cell;
    a.slotv[d] = base + (lane - hl);
  }
}

// ---------------------------------------------------------------- exclusive scan of counts
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_TILE = SCAN_ITEMS * SCAN_THREADS;

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Block-local exclusive scan of a tile of SCAN_TILE counts; the tile total goes to bsum[b].  The
// counts are zeroed once read (the histogram of the next build starts from zero).
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_local(int32_t *in, int64_t n, int32_t *out, int32_t *bsum) {
  __shared__ int wsum[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int tsum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    tsum += v[k];
  }
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) in[base + k] = 0;
  const int incl = wave_incl_scan(tsum);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int woff = 0;
  for (int k = 0; k < w; ++k) woff += wsum[k];
  int run = woff + incl - tsum;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == SCAN_THREADS - 1) bsum[blockIdx.x] = woff + incl;
}

// Exclusive scan of the nb tile totals in place (one block of TOP_THREADS, TOP_ITEMS consecutive
// totals per thread, sequential over chunks of TOP_TILE: one chunk up to 4096 tiles, i.e. 4 M
// bins), total to out[n] (and to out2[n2] when given).
constexpr int TOP_THREADS = 1024;
constexpr int TOP_ITEMS = 4;
constexpr int TOP_TILE = TOP_THREADS * TOP_ITEMS;
__global__ __launch_bounds__(TOP_THREADS) void k_scan_top(int32_t *bsum, int64_t nb, int32_t *out, int64_t n,
                                                          int32_t *out2, int64_t n2) {
  __shared__ int wsum[TOP_THREADS / 64];
  __shared__ int carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t c0 = 0; c0 < nb; c0 += TOP_TILE) {
    const int64_t base = c0 + (int64_t)threadIdx.x * TOP_ITEMS;
    int v[TOP_ITEMS];
    int tsum = 0;
#pragma unroll
    for (int k = 0; k < TOP_ITEMS; ++k) {
      v[k] = base + k < nb ? bsum[base + k] : 0;
      tsum += v[k];
    }
    const int incl = wave_incl_scan(tsum);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    // offsets of the waves: an inclusive scan of the 16 wave totals in the first lanes
    const int wt = lane < TOP_THREADS / 64 ? wsum[lane] : 0;
    const int wincl = wave_incl_scan(wt);
    const int woff = __shfl(wincl, w, 64) - __shfl(wt, w, 64);
    const int carry = carry_s;
    int run = carry + woff + incl - tsum;
#pragma unroll
    for (int k = 0; k < TOP_ITEMS; ++k) {
      if (base + k < nb) bsum[base + k] = run;
      run += v[k];
    }
    __syncthreads();
    if (threadIdx.x == TOP_THREADS - 1) carry_s = carry + woff + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[n] = carry_s;
    if (out2) out2[n2] = carry_s;
  }
}

// ---------------------------------------------------------------- stable placement + gather
// Bin start = tile-local prefix + scanned tile total: thread t < nbin writes start[t] (and, with
// half-edge cells, the cell start cstart[t / 8] from every eighth bin); visiting position t < N
// places its molecule at its provisional slot of its bin (both read only lstart and bsum).
__global__ __launch_bounds__(256) void k_scatter(const int32_t *cellv, const int32_t *slotv, const int32_t *order,
                                                 const int32_t *lstart, const int32_t *bsum, int64_t N, int64_t nbin,
                                                 int32_t *start, int32_t *cstart, int32_t *tmp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nbin) {
    const int32_t v = lstart[t] + bsum[t / SCAN_TILE];
    start[t] = v;
    if (cstart && (t & 7) == 0) cstart[t >> 3] = v;
  }
  if (t < N) {
    const int c = cellv[t];
    tmp[lstart[c] + bsum[c / SCAN_TILE] + slotv[t]] = order ? order[t] : (int32_t)t;
  }
}

// The caller-order cell ids of the view: cell_of[order[d]] = cellv[d] (its bin, shifted right by
// 3 when the bins are half-edge cells).
__global__ void k_cell_of(const int32_t *cellv, const int32_t *order, int64_t N, int shift, int32_t *cell_of) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d < N) cell_of[order ? order[d] : d] = cellv[d] >> shift;
}

struct GatherArgs {
  const double *pos, *quat;
  const int32_t *comp, *cellv, *start, *tmp, *order;
  int64_t N;
  double Lx, Ly, Lz;
  const ModelDev *md;
  int32_t sl, sc, sd, sq, nvec;
  int32_t *perm, *scomp;
  double *sx, *sy, *sz, *svec, *squat;
};

__device__ __forceinline__ void rotate(const double q[4], const double v[3], double o[3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  o[0] = (w * w + x * x - y * y - z * z) * v[0] + 2.0 * (x * y - w * z) * v[1] + 2.0 * (x * z + w * y) * v[2];
  o[1] = 2.0 * (x * y + w * z) * v[0] + (w * w - x * x + y * y - z * z) * v[1] + 2.0 * (y * z - w * x) * v[2];
  o[2] = 2.0 * (x * z - w * y) * v[0] + 2.0 * (y * z + w * x) * v[1] + (w * w - x * x - y * y + z * z) * v[2];
}

// Final position of molecule i inside its bin = number of molecules of the same bin with a
// smaller original index (a stable counting sort whatever order the atomic slots came in); then
// gather the sorted copies.  The bin's entries are contiguous in tmp, so the ranking reads
// cached words only.  Thread d takes molecule order[d] (identity without an order): in the
// previous build's order the sorted copies are written nearly in sequence.  The blocks of each
// XCD (block b runs on XCD b % 8) take one contiguous eighth of that order, so the COM lines a
// region of space gathers meet in one L2 instead of being fetched by several.
__global__ __launch_bounds__(256) void k_rank_gather(GatherArgs a) {
  const int64_t dd = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (dd >= a.N) return;
  const int64_t i = a.order ? (int64_t)a.order[dd] : dd;
  const int c = a.cellv[dd];
  const int s = a.start[c], n = a.start[c + 1] - s;
  int rank = 0;
  for (int k = 0; k < n; ++k) rank += a.tmp[s + k] < (int32_t)i ? 1 : 0;
  const int d = s + rank;
  a.perm[d] = (int32_t)i;
  double x = a.pos[3 * i], y = a.pos[3 * i + 1], z = a.pos[3 * i + 2];
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) x = y = z = __builtin_nan("");
  a.sx[d] = wrap1(x, a.Lx);
  a.sy[d] = wrap1(y, a.Ly);
  a.sz[d] = wrap1(z, a.Lz);
  int ci = 0;
  if (a.comp) {
    ci = a.comp[i];
    if (ci < 0 || ci >= a.md->ncomp) ci = 0;
  }
  if (a.scomp) a.scomp[d] = ci;
  if (a.svec) {
    const CompDev &cd = a.md->comp[ci];
    double q[4] = {1.0, 0.0, 0.0, 0.0};
    if (a.quat)
      for (int k = 0; k < 4; ++k) q[k] = a.quat[4 * i + k];
    for (int k = 0; k < 4; ++k) a.squat[4 * d + k] = q[k];
    double *out = a.svec + (int64_t)d * a.nvec * 3;
    double o[3];
    const double zero[3] = {0.0, 0.0, 0.0};
    int v = 0;
    for (int k = 0; k < a.sl; ++k, ++v) {
      rotate(q, k < cd.n_lj ? cd.lj_pos[k] : zero, o);
      out[3 * v] = o[0], out[3 * v + 1] = o[1], out[3 * v + 2] = o[2];
    }
    for (int k = 0; k < a.sc; ++k, ++v) {
      rotate(q, k < cd.n_chg ? cd.chg_pos[k] : zero, o);
      out[3 * v] = o[0], out[3 * v + 1] = o[1], out[3 * v + 2] = o[2];
    }
    for (int k = 0; k < a.sd; ++k, ++v) {
      rotate(q, k < cd.n_dip ? cd.dip_pos[k] : zero, o);
      out[3 * v] = o[0], out[3 * v + 1] = o[1], out[3 * v + 2] = o[2];
    }
    for (int k = 0; k < a.sd; ++k, ++v) {
      rotate(q, k < cd.n_dip ? cd.dip_dir[k] : zero, o);
      out[3 * v] = o[0], out[3 * v + 1] = o[1], out[3 * v + 2] = o[2];
    }
    for (int k = 0; k < a.sq; ++k, ++v) {
      rotate(q, k < cd.n_quad ? cd.quad_pos[k] : zero, o);
      out[3 * v] = o[0], out[3 * v + 1] = o[1], out[3 * v + 2] = o[2];
    }
    for (int k = 0; k < a.sq; ++k, ++v) {
      rotate(q, k < cd.n_quad ? cd.quad_dir[k] : zero, o);
      out[3 * v] = o[0], out[3 * v + 1] = o[1], out[3 * v + 2] = o[2];
    }
  }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_scale_copy(const double *src, double *dst, int64_t n, double a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = a * src[i];
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int launch_cell_of(const md_cells *c, hipStream_t s) {
  k_cell_of<<<nblk(c->N, 256), 256, 0, s>>>(c->cellv, c->order, c->N, c->sub ? 3 : 0, c->cell_of);
  return check_hip(hipGetLastError(), "k_cell_of");
}

int launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return MD_OK;
  k_fill_i32<<<nblk(n, 256), 256, 0, s>>>(p, n, v);
  return check_hip(hipGetLastError(), "k_fill_i32");
}

int launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return MD_OK;
  k_fill_f64<<<nblk(n, 256), 256, 0, s>>>(p, n, v);
  return check_hip(hipGetLastError(), "k_fill_f64");
}

int launch_scale_copy(const double *src, double *dst, int64_t n, double a, hipStream_t s) {
  if (n <= 0) return MD_OK;
  k_scale_copy<<<nblk(n, 256), 256, 0, s>>>(src, dst, n, a);
  return check_hip(hipGetLastError(), "k_scale_copy");
}

int launch_build(md_model *m, md_cells *c, const double *pos, const double *quat, const int32_t *comp, int64_t N,
                 const double inv_h[3], const double inv_hh[3], const int32_t *order, hipStream_t s) {
  int rc;
  // the histogram must start at zero: left so by the previous build's scan, else cleared here
  // (whole allocation, so a later build with more bins also starts from zero)
  if (!c->counts_zero && (rc = launch_fill_i32(c->count, c->cap_cell, 0, s))) return rc;
  c->counts_zero = false;
  const int64_t nbin = c->sub ? 8 * c->ncell : c->ncell;
  BinArgs b{pos,       quat,      comp,      order,     N,         c->box[0],     c->box[1],
            c->box[2], inv_h[0],  inv_h[1],  inv_h[2],  inv_hh[0], inv_hh[1],     inv_hh[2],
            c->nc[0],  c->nc[1],  c->nc[2],  m->host.ncomp, (int32_t)((m->flags & MD_CHECK) != 0), (int32_t)c->sub,
            c->cellv,  c->slot,   c->count,  m->status};
  k_bin<<<(unsigned)pair_blocks(nblk(N, 256)), 256, 0, s>>>(b);
  if ((rc = check_hip(hipGetLastError(), "k_bin"))) return rc;
  const int64_t nb = (nbin + SCAN_TILE - 1) / SCAN_TILE;
  k_scan_local<<<(unsigned)nb, SCAN_THREADS, 0, s>>>(c->count, nbin, c->lstart, c->bsum);
  k_scan_top<<<1, TOP_THREADS, 0, s>>>(c->bsum, nb, c->start, nbin, c->sub ? c->cstart : nullptr, c->ncell);
  if ((rc = check_hip(hipGetLastError(), "k_scan"))) return rc;
  c->counts_zero = true;
  k_scatter<<<nblk(std::max<int64_t>(N, nbin), 256), 256, 0, s>>>(c->cellv, c->slot, order, c->lstart, c->bsum, N,
                                                                   nbin, c->start, c->sub ? c->cstart : nullptr,
                                                                   c->tmp);
  if ((rc = check_hip(hipGetLastError(), "k_scatter"))) return rc;
  GatherArgs g{pos, m->single_site ? nullptr : quat, comp, c->cellv, c->start, c->tmp, order, N,
               c->box[0], c->box[1], c->box[2], m->dev, m->shape.lj, m->shape.chg, m->shape.dip, m->shape.quad,
               c->nvec, c->perm, m->single_site ? nullptr : c->scomp, c->sx, c->sy, c->sz,
               m->single_site ? nullptr : c->svec, m->single_site ? nullptr : c->squat};
  k_rank_gather<<<(unsigned)pair_blocks(nblk(N, 256)), 256, 0, s>>>(g);
  return check_hip(hipGetLastError(), "k_rank_gather");
}

}  // namespace mdcell
