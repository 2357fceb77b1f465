// Internal declarations shared by the libmdcell translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/md.h"

namespace mdcell {

// Site kinds as compile-time tags.
enum Kind : int { KIND_CHG = 1, KIND_DIP = 2, KIND_QUAD = 3 };

// Per-molecule vector slots of the sorted site arrays: LJ offsets, charge offsets, dipole
// offsets, dipole axes, quadrupole offsets, quadrupole axes, each group sized by the model's
// layout shape (SL, SC, SD, SQ).
struct Shape {
  int lj, chg, dip, quad;
  int nvec() const { return lj + chg + 2 * dip + 2 * quad; }
};

// One component as the kernels see it (FP64, body frame).
struct CompDev {
  int32_t n_lj, n_chg, n_dip, n_quad;
  int32_t rotates;  // any principal moment > 0
  int32_t pad_[3];
  double lj_pos[MD_MAX_LJ][3], lj_eps[MD_MAX_LJ], lj_sig[MD_MAX_LJ];
  double chg_pos[MD_MAX_CHG][3], chg_q[MD_MAX_CHG];
  double dip_pos[MD_MAX_DIP][3], dip_dir[MD_MAX_DIP][3], dip_mu[MD_MAX_DIP];
  double quad_pos[MD_MAX_QUAD][3], quad_dir[MD_MAX_QUAD][3], quad_Q[MD_MAX_QUAD];
  double mass, inv_mass, inertia[3], inv_inertia[3];
};

// LJ parameters of one site pair (a of component A, b of component B) after mixing, plus the
// adjoint's factors: pe = 1 / (2 eps_a) (d eps_ab / d eps_a = eps_ab pe, and u is linear in
// eps_ab), ps = (eta_AB / 2) 4 eps_ab / sigma_ab, csh = 12 (sigma_ab/r_c)^12 - 6 (sigma_ab/r_c)^6
// when shifted (else 0): du/dsigma_a = ps (12 s^12 - 6 s^6 - csh).
struct LJPair {
  double eps4, eps24, sig2, shift, pe, ps, csh, pad_;
};

struct ModelDev {
  int32_t ncomp, lj_shift;
  int32_t sl, sc, sd, sq;  // layout shape of the sorted site vectors
  double rc, rc2, kappa, kappa_rc3;  // kappa_rc3 = kappa / rc^3
  double xi[MD_MAX_COMP][MD_MAX_COMP], eta[MD_MAX_COMP][MD_MAX_COMP];
  CompDev comp[MD_MAX_COMP];
  LJPair lj[MD_MAX_COMP][MD_MAX_COMP][MD_MAX_LJ][MD_MAX_LJ];
  // sum of the LJTS shifts u_ab(r_c) over all LJ site pairs of a component pair: subtracted once
  // per interacting molecule pair in FP64 (a per-pair rounded constant would bias U)
  double shift_sum[MD_MAX_COMP][MD_MAX_COMP];
  int32_t param_off[MD_MAX_COMP];  // first parameter-gradient column of each component
  int32_t nparam;
};

// Everything a pair kernel needs about the sorted configuration.
struct CellsDev {
  const int32_t *cell_start, *perm, *scomp;
  // with half-edge cells: first sorted slot of half-cell 8 c + octant (octant 4 z + 2 y + x),
  // [8 ncell + 1]; else NULL
  const int32_t *sub_start;
  const double *sx, *sy, *sz;  // wrapped COMs in sorted order
  const double *svec;          // [N][nvec][3] world-frame site offsets / axes, sorted order
  const double *squat;         // [N][4] quaternions in sorted order (multi-site models), or NULL
  int32_t nx, ny, nz, ncell, nvec;
  double Lx, Ly, Lz, hx, hy, hz;
};


struct PairOut {
  double *force, *torque, *u_mol, *w_mol;
  int32_t *nnb_mol;
  double *partial;  // [gridDim.x][PARTIAL_COLS]
  // half-shell kernel: per-molecule rows in sorted order, row 0 the molecule's own sums, row
  // 1 + k the partner sums from the cell at half-stencil entry -k, summed by the gather:
  // rows [N3_ROWS][N][NT] force (NT = 3, one LJ site at the centre) or force and torque (NT = 6)
  // in the precision of the path (float or double), rows_uw [N3_ROWS][N][3] u, w and the partner
  // count in FP64 when nq = 9 (per-molecule outputs wanted; else nq = 6)
  void *rows;
  double *rows_uw;
  int64_t n;
  int nq;
  int32_t *status;
  // partner rows whose terms left the range of the exact LDS sums: bad[0] the count, bad[1 + e]
  // the row entry (row index x n + sorted molecule index), re-evaluated in FP64 by the fix-up
  unsigned long long *bad;
};
constexpr int BAD_CAP = 65536;
constexpr int PARTIAL_COLS = 5;  // u, wxx, wyy, wzz, nnb (the sum of nnb_mol: twice the pair count)
constexpr int N3_ROWS = 15;

struct AdjOut {
  double gU;
  double *dpos, *dquat;
  double *pgrad;  // [nblocks][nparam] per-block parameter partials (or nullptr)
};

}  // namespace mdcell

// Library-owned objects behind the opaque handles.
struct md_cells {
  int64_t N = 0, cap_N = 0;
  int64_t ncell = 0, cap_cell = 0, cap_blocks = 0;
  int32_t nc[3] = {0, 0, 0};
  double box[3] = {0, 0, 0};
  int nvec = 0, cap_nvec = 0;
  bool built = false;
  const md_model *model = nullptr;
  int32_t *cell_of = nullptr, *slot = nullptr, *tmp = nullptr, *perm = nullptr, *scomp = nullptr;
  // cell id at each position of the last build's visiting order (slot: provisional slot, same
  // order), and that order (NULL: index order; else perm_prev); cell_of (caller order, for
  // md_cells_view) is formed from them on demand
  int32_t *cellv = nullptr;
  const int32_t *order = nullptr;
  bool cell_of_valid = false;
  int32_t *perm_prev = nullptr;  // the other buffer of the permutation pair (previous build's order)
  // counting-sort bins: the cells, or with half-edge cells (sub) the 8 half-cells of each cell
  // (bin 8 c + octant); start has one entry per bin plus the total, cstart the cell starts then
  bool sub = false;
  int32_t *cstart = nullptr;
  int64_t cap_cstart = 0;
  int32_t *count = nullptr, *start = nullptr, *bsum = nullptr;
  int32_t *lstart = nullptr;     // tile-local exclusive prefix of the counts
  bool counts_zero = false;      // every entry of the count allocation is zero (left so by the scan)
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *svec = nullptr;
  // quaternions of the last build in sorted order (multi-site models): the adjoint's dU/dq
  // chain rule reads these, so it never depends on the caller's array after the build
  double *squat = nullptr;
  int64_t cap_squat = 0;
};

struct md_model {
  mdcell::ModelDev host;        // host copy of the device tables
  mdcell::ModelDev *dev = nullptr;
  mdcell::Shape shape{1, 0, 0, 0};
  bool single_site = true;      // one component, one LJ site at the COM
  bool fixed_shape = false;     // one component whose shape has a compiled kernel
  int64_t nparam = 0;
  std::vector<int64_t> param_off;  // per component offset into the parameter vector
  uint32_t flags = 0;
  int32_t *status = nullptr;    // device status word
  double *partial = nullptr;    // pair-kernel block partials
  int64_t cap_partial = 0;
  double *rows = nullptr;       // half-shell per-molecule rows (multi-site)
  int64_t cap_rows = 0;
  unsigned long long *bad = nullptr;  // [1 + BAD_CAP] rows for the FP64 fix-up (count first)
  double *red2 = nullptr;       // second-stage reduction buffer
  double *pgrad = nullptr;      // adjoint parameter partials
  int64_t cap_pgrad = 0;
  // md_step scratch; uw[8..15]: U, W, W_xx, W_yy, W_zz, K_trans, K_rot, rotational dof of a step
  double *force = nullptr, *torque = nullptr, *uw = nullptr;
  int64_t cap_step = 0;
  double T_target = 0.0;        // velocity-rescaling thermostat (0: NVE)
  // md_step with an energies row and no thermostat: each step's reduction runs on a side stream
  // (default priority), overlapping the next step; the partial rows alternate between two slots
  hipStream_t side = nullptr;
  hipEvent_t ev_leap[2] = {nullptr, nullptr}, ev_red[2] = {nullptr, nullptr};
  int lds_limit = 0;            // LDS bytes per block on the model's device (queried at first use)
  int lds_per_cu = 0;           // LDS bytes per CU (queried at first use)
  int lj1_static_lds[4] = {-1, -1, -1, -1};  // static LDS of the single-site pair kernel (FP64, FP32;
                                             // then with half-edge cells)
  // profiling
  bool profiling = false;
  struct Ev {
    int group;
    hipEvent_t a, b;
  };
  std::vector<Ev> events;
  double prof_ms[4] = {0, 0, 0, 0};
  int64_t prof_n[4] = {0, 0, 0, 0};
  hipStream_t last_stream = nullptr;
};

namespace mdcell {

// error plumbing (md_api.cpp)
int set_error(int code, const std::string &msg);
int check_hip(hipError_t e, const char *what);

// profiling helpers (md_api.cpp)
enum ProfGroup { PROF_PAIR = 0, PROF_BUILD = 1, PROF_STEP = 2, PROF_ADJ = 3 };
void prof_begin(md_model *m, int group, hipStream_t s, hipEvent_t *a);
void prof_end(md_model *m, int group, hipStream_t s, hipEvent_t a);

// launchers
int launch_build(md_model *m, md_cells *c, const double *pos, const double *quat, const int32_t *comp, int64_t N,
                 const double inv_h[3], const double inv_hh[3], const int32_t *order, hipStream_t s);
int launch_pair(md_model *m, const md_cells *c, int precision, const PairOut &o, hipStream_t s, int64_t *nblocks);
int launch_reduce(md_model *m, int64_t nrows, int ncols, const double *rows, double *out, hipStream_t s);
// pair partial rows -> uw[0..4] (U, W, W_aa), pair count, energies row; with kin_rows (the
// leapfrog's [kin_nrows][KIN_COLS] partials) also K_trans and K_rot of the energies row and
// uw[5..7] = K_trans, K_rot, rotational degrees of freedom
int launch_reduce_forces(md_model *m, int64_t nrows, const double *rows, double *uw, int64_t *npairs,
                         double *energies_row, hipStream_t s, const double *kin_rows = nullptr,
                         int64_t kin_nrows = 0);
constexpr int KIN_COLS = 3;  // K_trans, K_rot, rotational degrees of freedom
// velocity rescaling to the kinetic temperature T_target from the reduced kin[0..2]
int launch_rescale(md_model *m, double *vel, double *angmom, const int32_t *comp, int64_t N, const double *kin,
                   double T_target, hipStream_t s);
// leapfrog step; writes its kinetic-energy partial rows ([*kin_nrows][KIN_COLS]) to kin_rows
int launch_leapfrog(md_model *m, double *pos, double *vel, double *quat, double *angmom, const int32_t *comp,
                    int64_t N, const double box[3], double dt, const double *force, const double *torque,
                    double *kin_rows, int64_t *kin_nrows, hipStream_t s);
int launch_adjoint(md_model *m, const md_cells *c, int precision, const AdjOut &o, const double *quat,
                   hipStream_t s, int64_t *nblocks);
// single-site LJ adjoint after the force kernel: dpos = -gU F in place; dparams[0..4] (NULL
// allowed) from U, W (uw[0], uw[1]) and the pair count
int launch_lj_adjoint_finish(const md_model *m, double *dpos, int64_t N, double gU, const double *uw,
                             const int64_t *npairs, double *dparams, hipStream_t s);
// device address of the static scratch array of md_forces_noalloc on the current device (looked
// up once per device with hipGetSymbolAddress; md_pair.hip)
int noalloc_scratch(void **ptr);
int launch_cell_of(const md_cells *c, hipStream_t s);  // cell_of[order[d]] = cellv[d]
int launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
int launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
int launch_scale_copy(const double *src, double *dst, int64_t n, double a, hipStream_t s);

// number of pair-kernel blocks for a grid of ncell cells (a multiple of 8, see xcd_remap)
inline int64_t pair_blocks(int64_t ncell) { return ((ncell + 7) / 8) * 8; }

}  // namespace mdcell

// Periodic wrap into [0, L): x - L floor(x / L), minus L once more if rounding left it at L.
// The library is compiled without floating-point contraction, so this is one division, one
// floor, one multiply and one subtraction, each correctly rounded.
__device__ __forceinline__ double wrap1(double x, double L) {
  double xw = x - L * floor(x / L);
  if (xw >= L) xw -= L;
  return xw;
}

// Blocks of one launch are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8),
// each XCD with its own L2.  Give XCD k a contiguous run of cells so that neighbouring cells,
// which read the same neighbour data, meet in one L2.  nblocks is a multiple of 8.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int per = nblocks >> 3;
  return (b & 7) * per + (b >> 3);
}
