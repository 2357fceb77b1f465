/*
 * md.h -- C ABI of libmdcell: linked-cell short-range forces for rigid multi-centre molecules
 * on AMD Instinct MI355X (gfx950).
 *
 * Problem statement (ls1 mardyn, Niethammer et al., JCTC 2014):
 *   - molecules are rigid rotators: a centre of mass (COM) and an orientation quaternion, no
 *     internal degrees of freedom (Sec. 2, first paragraph; quaternions in Sec. 3, Eqs. 4-5);
 *   - interaction sites per molecule type: Lennard-Jones 12-6 sites (Sec. 2, LJ equation),
 *     optionally truncated and shifted (LJTS), Lorentz-Berthelot mixing with binary interaction
 *     parameters; point charges, point dipoles and linear point quadrupoles (Sec. 2, multipole
 *     paragraph), units with k_B = k_C = 1 (Sec. 2, Table 1);
 *   - reaction field for dipoles (Sec. 3, second paragraph);
 *   - neighbour search with linked cells of edge >= r_c and periodic boundaries (Sec. 3,
 *     linked-cell paragraphs); the cutoff acts on the COM distance;
 *   - per-molecule forces and torques by summation over pairs (Sec. 3, after Fig. 1);
 *   - leapfrog integration of translation and quaternion rotation (Sec. 3, Eqs. 2-5).
 *
 * Conventions for every entry point:
 *   - Arrays are DEVICE pointers (hipMalloc'd or a torch CUDA tensor's data_ptr()) unless the
 *     comment says "host".  All device arrays are dense, row-major, FP64 unless typed otherwise.
 *   - Calls that take `stream` (a hipStream_t, NULL = the legacy default stream) enqueue work on
 *     it and return without synchronising, except where a comment says "syncs".
 *   - Every call returns MD_OK (0) or a negative MD_E* code; the thread-local text of the last
 *     failure is returned by md_last_error().  No exception or abort crosses the ABI.
 *   - Host-checkable errors (NULL pointers, sizes, box too small) are reported synchronously
 *     before anything is enqueued.  Errors only the device can see (non-finite coordinates,
 *     component ids out of range, non-unit quaternions) raise bits of a device status word that
 *     md_status() reads (syncs); with MD_CHECK in the model flags every call syncs and checks it.
 *   - Quaternions are scalar-first (w, x, y, z) and rotate body-frame vectors into the space
 *     frame with the polynomial matrix A(q) (no normalisation inside); gradients with respect
 *     to quaternions are taken with respect to the four raw components.
 *   - Output arrays indexed by molecule are written in the caller's ORIGINAL molecule order.
 *   - One md_model (and the md_cells used with it) per stream at a time; calls on one model from
 *     several host threads must be serialised by the caller.
 */
#ifndef MDCELL_MD_H
#define MDCELL_MD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MD_OK = 0,
  MD_EINVAL = -1,      /* NULL required pointer, N <= 0, r_c <= 0, bad precision, bad table */
  MD_EBOX = -2,        /* a box side holds fewer than three cells of edge > r_c */
  MD_ECOMP = -3,       /* component table exceeds the compiled limits below */
  MD_ENONFINITE = -4,  /* non-finite host argument (box, r_c, dt, table entry) */
  MD_EHIP = -5,        /* HIP runtime error; text in md_last_error() */
  MD_ENOMEM = -6,      /* device allocation failed */
  MD_EDEVICE = -7      /* device status word non-zero (only with MD_CHECK or md_status) */
};

/* md_model_create flags */
#define MD_LJ_SHIFT 0x1u /* LJTS: subtract u_ab(r_c) from every LJ site pair inside the cutoff */
#define MD_CHECK 0x2u    /* validate inputs on the device and sync after every call */
#define MD_HALF_SHELL 0x4u /* single-site models: evaluate each molecule pair once (Newton's third
                              law, Fig. 1) with exact partner sums, as multi-site models always do.
                              Faster for strongly uneven cell occupancy (a vapour-liquid slab),
                              slower for homogeneous fluids; results differ from the default
                              kernel by rounding only.  No effect on multi-site models. */
#define MD_SUBCELLS 0x8u /* single-site models without MD_HALF_SHELL: sort the molecules of each
                            cell by half-edge (r_c/2) cell (Sec. 3) and skip, in the cutoff walk,
                            the far z-half of the cell layer above or below a molecule's own
                            z-half, which lies more than one cell edge (>= r_c) away.  The pair set
                            is unchanged, the results differ by rounding only;
                            md_cells_info.sub_start gives the half-edge cell ranges. */

/* precision argument */
#define MD_FP64 0 /* all pair arithmetic and accumulation in FP64 */
#define MD_FP32 1 /* single-site LJ: cutoff test in FP32 with a proven guard band, every listed
                     pair decided exactly in FP64 (the pair set is the FP64 one), force and virial
                     in FP32, per-molecule sums cascaded from FP32 into FP64.  Multi-site:
                     reciprocals seeded in FP32, multipole terms in FP32; COM test, LJ site
                     separations, LJ terms and pair energies in FP64.  Energies, accumulation
                     across flushes and all reductions in FP64. */

/* device status word bits (md_status) */
#define MD_DEV_NONFINITE 0x1 /* a position was NaN/Inf: that molecule is spread into cell
                                (index mod ncell), takes part in no pair and gets zero force,
                                torque and energy; the others are evaluated as without it */
#define MD_DEV_COMP 0x2      /* a component id was outside [0, ncomp) */
#define MD_DEV_QUAT 0x4      /* | |q|^2 - 1 | > 1e-6 for some molecule */
#define MD_DEV_CAPACITY 0x8  /* internal capacity exceeded (should not happen) */
#define MD_DEV_RANGE 0x10    /* multi-site: more than 65 536 partner sums had a pair term beyond the
                                range of the exact LDS sums (2^24 FP32, 2^23 FP64: overlapping
                                molecules) and needed the FP64 fix-up; the force and torque of
                                the partners beyond that number are NaN */

/* compiled limits of the component table */
#define MD_MAX_COMP 4
#define MD_MAX_LJ 4
#define MD_MAX_CHG 4
#define MD_MAX_DIP 2
#define MD_MAX_QUAD 2

/* One rigid molecule type (host memory, body frame: COM at the origin, principal axes = body
 * axes).  LJ sites meet LJ sites only; charges, dipoles and quadrupoles meet each other. */
typedef struct {
  int32_t n_lj, n_chg, n_dip, n_quad;
  const double *lj_pos;   /* [n_lj][3] site offsets from the COM */
  const double *lj_eps;   /* [n_lj] epsilon_a > 0 */
  const double *lj_sigma; /* [n_lj] sigma_a > 0 */
  const double *chg_pos;  /* [n_chg][3] */
  const double *chg_q;    /* [n_chg] charge */
  const double *dip_pos;  /* [n_dip][3] */
  const double *dip_dir;  /* [n_dip][3] unit axis */
  const double *dip_mu;   /* [n_dip] dipole moment */
  const double *quad_pos; /* [n_quad][3] */
  const double *quad_dir; /* [n_quad][3] unit axis */
  const double *quad_Q;   /* [n_quad] linear quadrupole moment (phi = Q P2(cos theta) / r^3) */
  double mass;            /* > 0 */
  double inertia[3];      /* principal moments; 0 allowed (axis of a linear molecule) */
} md_component_desc;

typedef struct md_model md_model; /* opaque: device copy of the model tables + scratch */
typedef struct md_cells md_cells; /* opaque: cell grid + molecules sorted into cells */

/* Read-only view of a built cell grid (device pointers owned by the md_cells object, valid until
 * the next md_build_cells / md_cells_destroy on it).  md_cells_view forms cell_of on the device
 * on its first call after a build (syncs the model's last stream).  Cells have edge h_k = L_k / n_k > r_c,
 * n_k = floor(L_k / r_c) reduced until h_k >= r_c (1 + 2^-30); linear cell id
 * (c_z n_y + c_y) n_x + c_x.  Molecules are sorted stably by cell: within a cell by original
 * index, or with MD_SUBCELLS by half-edge cell s_k = min(2 n_k - 1, floor(x_w * (2 n_k / L_k)))
 * (octant 4 (s_z mod 2) + 2 (s_y mod 2) + (s_x mod 2)), then by original index. */
typedef struct {
  int64_t N;
  int64_t ncell;
  int32_t nc[3];
  double box[3];
  const int32_t *cell_of;    /* [N] cell of each molecule, original order */
  const int32_t *cell_start; /* [ncell + 1] first sorted slot of each cell */
  const int32_t *perm;       /* [N] original index of the molecule in each sorted slot */
  const int32_t *sub_start;  /* [8 ncell + 1] with MD_SUBCELLS: first sorted slot of half-edge cell
                              * 8 c + 4 z + 2 y + x (x, y, z the low bits of its half-cell
                              * coordinates) of cell c; else NULL */
} md_cells_info;

/* Create a model from ncomp host component descriptions (Sec. 2).  xi, eta: host
 * [ncomp][ncomp] Berthelot / Lorentz binary factors (symmetric), NULL for all ones: pair
 * epsilon_ab = xi_AB sqrt(eps_a eps_b), sigma_ab = eta_AB (sigma_a + sigma_b) / 2.  rc: COM
 * cutoff.  eps_rf: reaction-field permittivity, INFINITY allowed, applied to dipole-dipole site
 * pairs of molecule pairs inside the cutoff as -kappa mu_a.mu_b / r_c^3 with
 * kappa = 2 (eps_rf - 1) / (2 eps_rf + 1) (kappa = 1 at infinity).  flags: MD_LJ_SHIFT,
 * MD_CHECK, MD_HALF_SHELL, MD_SUBCELLS.  *out receives the model (owned by the caller, free with md_model_destroy).
 * Allocates device memory on the current device.  Errors: MD_EINVAL, MD_ECOMP, MD_ENONFINITE,
 * MD_ENOMEM, MD_EHIP. */
int md_model_create(const md_component_desc *comps, int32_t ncomp, const double *xi, const double *eta, double rc,
                    double eps_rf, uint32_t flags, md_model **out);
int md_model_destroy(md_model *m);

/* Number of doubles md_forces_adjoint writes to dparams, and the offset of each block:
 * for component c in order, for each LJ site [deps, dsigma, dx, dy, dz], then each charge
 * [dq, dx, dy, dz], each dipole [dmu, dx, dy, dz], each quadrupole [dQ, dx, dy, dz]
 * (dx, dy, dz: derivative w.r.t. the body-frame site offset). */
int64_t md_param_count(const md_model *m);

/* Read (get) or replace (set) the model's differentiable parameters, host [md_param_count(m)]
 * doubles in the layout of md_param_count and md_forces_adjoint's dparams: the site energies,
 * sizes, body-frame offsets, charges and dipole / quadrupole moments of Sec. 2's models.  set
 * re-derives the mixed LJ pair tables (Lorentz-Berthelot with the model's xi / eta) and the LJTS
 * shifts, then waits for all work on the device (syncs) and uploads the tables; masses, inertia,
 * site axes, r_c and the reaction field are unchanged.  The site of a single-site model stays at
 * its centre of mass.  Errors: NULL argument (MD_EINVAL), non-finite value (MD_ENONFINITE), LJ
 * epsilon or sigma <= 0 or a moved single-site offset (MD_EINVAL; the model is unchanged),
 * MD_EHIP. */
int md_model_get_params(const md_model *m, double *params);
int md_model_set_params(md_model *m, const double *params);

int md_cells_create(md_cells **out);
int md_cells_destroy(md_cells *c);
int md_cells_view(const md_cells *c, md_cells_info *out);

/* Linked-cell build (Sec. 3, linked-cell paragraph; periodic boundaries): wrap every COM into
 * [0, L_k) as x - L floor(x / L) (minus L once more if rounding left it at L), assign cell
 * c_k = min(n_k - 1, floor(x_w * (n_k / L_k))), counting-sort the molecules stably into cells
 * and gather sorted structure-of-arrays copies: wrapped COMs, component ids and, for multi-site
 * models, world-frame site offsets A(q) d_a and axes A(q) e_a.
 *   pos  [N][3] COM positions (any real values; wrapped copies are taken)
 *   quat [N][4] orientations, or NULL if every component is a single site at its COM
 *   comp [N] component ids (int32), or NULL if ncomp == 1
 *   box  host [3] periodic box lengths
 * Grows the cells' buffers on demand (hipMalloc), otherwise allocation-free.  Errors: MD_EINVAL,
 * MD_EBOX, MD_ENONFINITE, MD_ENOMEM, MD_EHIP. */
int md_build_cells(md_model *m, md_cells *cells, const double *pos, const double *quat, const int32_t *comp,
                   int64_t N, const double box[3], void *stream);

/* Forces, torques, energy and virial of the built configuration (Sec. 3): every molecule pair
 * whose minimum-image COM distance r satisfies fma(dz,dz,fma(dy,dy,dx*dx)) < r_c*r_c
 * interacts through all its site pairs.
 *   precision MD_FP64 or MD_FP32
 *   force   [N][3]  sum of site forces on each molecule (required)
 *   torque  [N][3]  torque about the COM (NULL allowed; required content only for multi-site)
 *   u_mol   [N]     half of the pair energies of each molecule (NULL allowed)
 *   w_mol   [N]     half of the molecular virials r_ij . F_ij of each molecule (NULL allowed)
 *   nnb_mol [N]     int32 number of partners inside the cutoff (NULL allowed)
 *   uw      [5]     U, W, W_xx, W_yy, W_zz (required; FP64, deterministic fixed-order sums)
 *   npairs  [1]     int64 number of unordered interacting pairs (NULL allowed)
 * Results are bitwise reproducible run to run.  Errors: MD_EINVAL, MD_EHIP, MD_EDEVICE. */
int md_forces(md_model *m, const md_cells *cells, int precision, double *force, double *torque, double *u_mol,
              double *w_mol, int32_t *nnb_mol, double *uw, int64_t *npairs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): md_forces with its per-call scratch -- the pair
 * kernel's block partials and, for multi-site models and MD_HALF_SHELL, the per-molecule partner
 * rows -- in one static device array of MD_NOALLOC_SCRATCH_BYTES per GPU, held until the process
 * ends, instead of model-owned buffers.  Arguments, kernels and results are those of md_forces,
 * bit for bit.  It calls no hipMalloc / hipFree; the model's fixed tables (md_model_create) and
 * the cells (md_build_cells, which allocates only when they grow) are used as they are.  The
 * scratch needed is 40 bytes per cell and 1 byte per molecule (block partials) plus, for the
 * half-shell kernels, 15 partner rows per molecule: 180 B (single-site) or 360 B (multi-site) in
 * FP32, twice that in FP64, and 360 B more when u_mol, w_mol or nnb_mol is given.  A
 * configuration that needs more than the array returns MD_EINVAL with nothing enqueued: beyond
 * about 400 000 cells for single-site models without MD_HALF_SHELL, beyond about 23 000
 * molecules for multi-site FP32 with per-molecule outputs.
 * Every call on one GPU uses that GPU's one array: calls that overlap on one GPU (two streams,
 * two threads) race and give wrong results.  The array needs no clearing: every call overwrites
 * what it reads.  Errors as md_forces. */
#define MD_NOALLOC_SCRATCH_BYTES (16u << 20)
int md_forces_noalloc(md_model *m, const md_cells *cells, int precision, double *force, double *torque,
                      double *u_mol, double *w_mol, int32_t *nnb_mol, double *uw, int64_t *npairs, void *stream);

/* nsteps leapfrog steps (Sec. 3, Eqs. 2-5), each: build cells, forces/torques at t,
 *   v(t + dt/2) = v(t - dt/2) + dt F / m,  r(t + dt) = r(t) + dt v(t + dt/2)  (wrapped),
 * and for molecules with inertia, Fincham's rotational leapfrog with the space-frame angular
 * momentum j: j(t) = j(t - dt/2) + dt/2 tau;  q(t + dt/2) = normalise(q + dt/2 qdot(q, w(t)));
 * j(t + dt/2) = j(t - dt/2) + dt tau;  q(t + dt) = normalise(q + dt qdot(q(t + dt/2),
 * w(t + dt/2))), qdot(q, w) = q (x) (0, w_body) / 2, w_body = I^-1 A(q)^T j (I_k^-1 := 0 where
 * I_k = 0).  pos, vel [N][3], quat [N][4] (NULL for single-site models), angmom [N][3] (NULL
 * likewise) are updated in place.  energies [nsteps][4] (NULL allowed) receives per step
 * U(t), K_trans(t) (v(t) = mean of the half-step velocities), K_rot(t), W(t).  With energies
 * or a thermostat (and nsteps > 1), each step's reduction, and the thermostat's rescaling, run
 * on a stream owned by the model (default priority), ordered after the step by an event and
 * overlapping the next step's cell build and forces; the next leapfrog waits for them, and
 * before the call returns the caller's stream waits for the last of them, so every result is
 * ordered on the caller's stream as usual.  Errors as md_build_cells and md_forces. */
int md_step(md_model *m, md_cells *cells, double *pos, double *vel, double *quat, double *angmom,
            const int32_t *comp, int64_t N, const double box[3], double dt, int64_t nsteps, int precision,
            double *energies, void *stream);

/* NVT by velocity rescaling (Sec. 2: in NVT the temperature is kept constant by velocity
 * rescaling), applied by later md_step calls on this model (host call, no device work):
 *   T_target > 0  every step ends by multiplying the new half-step velocities v(t + dt/2) and,
 *                 for molecules with inertia, the angular momenta j(t + dt/2) by
 *                 beta = sqrt(T_target / T(t)),  T(t) = 2 (K_trans(t) + K_rot(t)) / f  (k_B = 1),
 *                 f = 3 N + the number of nonzero principal moments of every molecule with
 *                 inertia; K(t) as in the energies row, which keeps the values before rescaling
 *                 (beta = 1 when K(t) = 0);
 *   T_target = 0  NVE (the default).
 * Errors: NULL model or T_target < 0 (MD_EINVAL), T_target not finite (MD_ENONFINITE). */
int md_set_thermostat(md_model *m, double T_target);

/* Isotropic cut-off corrections of the potential energy and of the virial W = sum r_ij . F_ij
 * (Sec. 3: the long-range part of the dispersive interaction is a mean-field integral beyond
 * r_c).  Host-only: takes the component table as md_model_create does (host memory) and returns
 *   *u_lrc = sum_{A,B} sum_{a,b} 2 pi N_A N_B / V * 4 eps_ab (sigma_ab^12 / (9 r_c^9) - sigma_ab^6 / (3 r_c^3))
 *   *w_lrc = sum_{A,B} sum_{a,b} 2 pi N_A N_B / V * 4 eps_ab (4 sigma_ab^12 / (3 r_c^9) - 2 sigma_ab^6 / r_c^3)
 * over ordered component pairs (A, B) and their LJ sites (a, b), Lorentz-Berthelot mixing with
 * xi/eta, each site pair taken at the centre distance (the cutoff acts on the COM distance),
 * V = box[0] box[1] box[2], counts [ncomp] (host, >= 0) molecules per component.  With
 * MD_LJ_SHIFT in flags the truncated-shifted potential is the model and both are 0.  Charges,
 * dipoles (reaction field) and quadrupoles add nothing.
 * Errors: NULL argument or invalid table / count / box / r_c (MD_EINVAL, MD_ECOMP,
 * MD_ENONFINITE, as md_model_create). */
int md_long_range_correction(const md_component_desc *comps, int32_t ncomp, const double *xi, const double *eta,
                             double rc, uint32_t flags, const int64_t *counts, const double box[3], double *u_lrc,
                             double *w_lrc);

/* Gradient of gU * U for the built configuration, recomputing every pair (no stored pair list).
 * Single-site models take one force evaluation: dU/dr_i = -F_i, U is linear in eps, sigma dU/dsigma
 * is the virial W minus the shift's share, and the offset gradient sum_i dU/dr_i vanishes.
 * "The built configuration" is the library-owned copy that the last md_build_cells on `cells`
 * took of pos and quat (sorted COMs, quaternions and site vectors): the caller may change or free
 * its own pos / quat arrays after md_build_cells returns.  After md_step, that copy is the
 * configuration at the start of the last step (before its drift), not the updated arrays; build
 * again to differentiate the new state. */
/* Outputs:
 *   dpos    [N][3]  gU dU/dr_i (= -gU F_i)
 *   dquat   [N][4]  gU dU/dq_i with respect to the raw quaternion components (NULL allowed)
 *   dparams [md_param_count(m)] gU dU/d(parameters), layout as md_param_count (NULL allowed:
 *           the kernels then leave the parameter partials out of the pair loop, which makes a
 *           dpos / dquat-only call markedly cheaper)
 * The molecule-pair set is the one fixed by the cutoff (U is differentiated piecewise).
 * Errors: MD_EINVAL, MD_EHIP. */
int md_forces_adjoint(md_model *m, const md_cells *cells, int precision, double gU, double *dpos, double *dquat,
                      double *dparams, void *stream);

/* Synchronises the model's last stream, returns the device status word in *flags (host) and
 * clears it.  Returns MD_OK, or MD_EHIP. */
int md_status(md_model *m, int32_t *flags);

/* Kernel timing with HIP events recorded on the launch stream around the pair kernel and around
 * the cell build.  md_profile(m, 1) starts (and clears) recording; md_profile_read syncs and
 * returns the total milliseconds and launch counts of the pair kernels ("pair"), the cell
 * build ("build"), the leapfrog kernels ("step") and the adjoint kernels ("adjoint"). */
int md_profile(md_model *m, int enable);
int md_profile_read(md_model *m, const char *group, double *total_ms, int64_t *launches);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *md_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
