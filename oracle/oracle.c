/*
 * oracle.c -- plain FP64 brute-force reference for the linked-cell rigid-molecule force path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this file;
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What it computes (ls1 mardyn, Niethammer et al., JCTC 2014):
 *   - rigid rotators: centre of mass (COM) plus a quaternion orientation, no internal degrees of
 *     freedom (Sec. 2, first paragraph);
 *   - Lennard-Jones 12-6 sites (Sec. 2, LJ equation), optionally truncated and shifted (LJTS),
 *     Lorentz-Berthelot mixing with binary parameters xi/eta (Sec. 2, second paragraph);
 *   - point charges, point dipoles and linear point quadrupoles (Sec. 2, multipole paragraph),
 *     in units with k_C = 1 (Sec. 2, units paragraph and Table 1);
 *   - the reaction field for dipoles (Sec. 3, second paragraph), Barker-Watts form, applied to
 *     dipole-dipole site pairs of molecule pairs inside the cutoff;
 *   - the cutoff acts on the COM distance; cells have edge >= r_c (Sec. 3, linked-cell paragraph)
 *     and the box is periodic (Sec. 3, periodic-boundary sentence before Fig. 1);
 *   - per-molecule forces and torques obtained by summation over all pairs (Sec. 3, after Fig. 1);
 *   - the leapfrog integrator for translation and quaternion rotation (Sec. 3, Eqs. 2-5).
 *
 * The method (linked cells) reaches exactly the brute-force result, so this file is the plain
 * definition: for every molecule i, a loop over every other molecule j with the minimum image.
 * No cells, no blocking, no reordering.  Build with -ffp-contract=off; the one fused operation is
 * the explicit fma() nesting of the squared COM distance, which fixes the cutoff decision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Site kinds in the flat site table: one record of OM_SITE_STRIDE doubles per site:
 *   [kind, px, py, pz, ex, ey, ez, p0, p1, 0]
 *   kind 0: LJ site,        p0 = epsilon, p1 = sigma
 *   kind 1: point charge,   p0 = q
 *   kind 2: point dipole,   (ex,ey,ez) = unit axis, p0 = mu
 *   kind 3: lin. quadrupole,(ex,ey,ez) = unit axis, p0 = Q (Buckingham, phi = Q P2(cos)/r^3)
 * (px,py,pz) is the site offset from the COM in the body frame.                               */
#define OM_SITE_STRIDE 10
#define OM_LJ 0
#define OM_CHG 1
#define OM_DIP 2
#define OM_QUAD 3
#define OM_MAXSITE 16

typedef struct {
  int32_t ncomp;
  const int32_t *site_start; /* [ncomp+1] offsets into sites */
  const double *sites;       /* [nsites][OM_SITE_STRIDE] */
  const double *xi;          /* [ncomp*ncomp] Berthelot factor on epsilon */
  const double *eta;         /* [ncomp*ncomp] Lorentz factor on sigma */
  double rc;
  double eps_rf;             /* reaction-field permittivity; INFINITY allowed */
  int32_t lj_shift;          /* 1: truncated-shifted LJ (LJTS) */
} om_model;

/* ---------------------------------------------------------------- geometry helpers */

/* Body-to-space rotation matrix of q = (w, x, y, z), polynomial form (no normalisation). */
static void om_rotmat(const double *q, double A[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  A[0][0] = w * w + x * x - y * y - z * z;
  A[0][1] = 2.0 * (x * y - w * z);
  A[0][2] = 2.0 * (x * z + w * y);
  A[1][0] = 2.0 * (x * y + w * z);
  A[1][1] = w * w - x * x + y * y - z * z;
  A[1][2] = 2.0 * (y * z - w * x);
  A[2][0] = 2.0 * (x * z - w * y);
  A[2][1] = 2.0 * (y * z + w * x);
  A[2][2] = w * w - x * x - y * y + z * z;
}

static void om_matvec(const double A[3][3], const double *v, double *out) {
  for (int r = 0; r < 3; ++r) out[r] = A[r][0] * v[0] + A[r][1] * v[1] + A[r][2] * v[2];
}

static void om_matTvec(const double A[3][3], const double *v, double *out) {
  for (int c = 0; c < 3; ++c) out[c] = A[0][c] * v[0] + A[1][c] * v[1] + A[2][c] * v[2];
}

static void om_cross(const double *a, const double *b, double *out) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

static double om_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Gradient of g . (A(q) v) with respect to the four raw quaternion components, from
 * A(q) v = (w^2 - |u|^2) v + 2 (u.v) u + 2 w (u x v), q = (w, u).                              */
static void om_quat_grad(const double *q, const double *v, const double *g, double *dq) {
  const double w = q[0];
  const double u[3] = {q[1], q[2], q[3]};
  double uxv[3], vxg[3];
  om_cross(u, v, uxv);
  om_cross(v, g, vxg);
  const double gv = om_dot(g, v), gu = om_dot(g, u), uv = om_dot(u, v);
  dq[0] += 2.0 * w * gv + 2.0 * om_dot(g, uxv);
  for (int k = 0; k < 3; ++k) dq[1 + k] += -2.0 * gv * u[k] + 2.0 * gu * v[k] + 2.0 * uv * g[k] + 2.0 * w * vxg[k];
}

/* Cells per axis: floor(L / r_c), reduced until the cell edge exceeds r_c by a relative margin of
 * 2^-30, so that a pair inside the cutoff can never skip a cell through rounding of the bin
 * index.  Returns 0 if any axis has fewer than three cells.                                      */
int oracle_ncells(const double *box, double rc, int32_t *nc) {
  for (int k = 0; k < 3; ++k) {
    double n = floor(box[k] / rc);
    while (n >= 1.0 && box[k] / n < rc * (1.0 + 0x1p-30)) n -= 1.0;
    if (n < 3.0) return 0;
    nc[k] = (int32_t)n;
  }
  return 1;
}

/* Wrap one coordinate into [0, L): x - L floor(x / L), then subtract L once if rounding left it
 * at L.                                                                                          */
static double om_wrap(double x, double L) {
  double xw = x - L * floor(x / L);
  if (xw >= L) xw -= L;
  return xw;
}

/* Wrap + bin (periodic boundaries; cells of edge L/n >= r_c, linear index x fastest).
 * cell_of[i] = (cz * ny + cy) * nx + cx with ck = min(n_k - 1, floor(xw_k * (n_k / L_k))).
 * Returns the number of cells, or -1 if the box is too small for three cells per axis.          */
int64_t oracle_bin(const double *pos, int64_t N, const double *box, double rc, int32_t *cell_of, double *pos_w) {
  int32_t nc[3];
  if (!oracle_ncells(box, rc, nc)) return -1;
  double inv_h[3];
  for (int k = 0; k < 3; ++k) inv_h[k] = (double)nc[k] / box[k];
  for (int64_t i = 0; i < N; ++i) {
    int32_t c[3];
    for (int k = 0; k < 3; ++k) {
      const double xw = om_wrap(pos[3 * i + k], box[k]);
      if (pos_w) pos_w[3 * i + k] = xw;
      double f = floor(xw * inv_h[k]);
      int32_t ck = (int32_t)f;
      if (ck > nc[k] - 1) ck = nc[k] - 1;
      if (ck < 0) ck = 0;
      c[k] = ck;
    }
    cell_of[i] = (c[2] * nc[1] + c[1]) * nc[0] + c[0];
  }
  return (int64_t)nc[0] * nc[1] * nc[2];
}

/* Half-edge cells (Sec. 3, the r_c/2 variant of the linked cells): the grid of 2 n_k cells of
 * edge L_k / (2 n_k) per axis, after the same wrap as oracle_bin.  half_of[3 i + k] =
 * min(2 n_k - 1, floor(xw_k * (2 n_k / L_k))).  Each edge-r_c cell of oracle_bin is made of the
 * 2 x 2 x 2 half-edge cells whose indices halved (integer division) are its cell coordinates.
 * Returns 8 x the number of edge-r_c cells, or -1 if the box is too small for three cells per
 * axis.                                                                                          */
int64_t oracle_half_cells(const double *pos, int64_t N, const double *box, double rc, int32_t *half_of) {
  int32_t nc[3];
  if (!oracle_ncells(box, rc, nc)) return -1;
  double inv_hh[3];
  for (int k = 0; k < 3; ++k) inv_hh[k] = (double)(2 * nc[k]) / box[k];
  for (int64_t i = 0; i < N; ++i) {
    for (int k = 0; k < 3; ++k) {
      const double xw = om_wrap(pos[3 * i + k], box[k]);
      int32_t s = (int32_t)floor(xw * inv_hh[k]);
      if (s > 2 * nc[k] - 1) s = 2 * nc[k] - 1;
      if (s < 0) s = 0;
      half_of[3 * i + k] = s;
    }
  }
  return 8 * (int64_t)nc[0] * nc[1] * nc[2];
}

/* ---------------------------------------------------------------- one site pair */

/* Energy and partial derivatives of one electrostatic site pair, as a function of the distance r
 * and the three cosines c_i = e_a.rhat, c_j = e_b.rhat, c_ij = e_a.e_b (rhat points from site b
 * of molecule j to site a of molecule i).  Multipole forms of the point-charge / point-dipole /
 * linear-quadrupole expansion (k_C = 1); kappa is the reaction-field factor for dipole pairs.   */
typedef struct { double u, ur, uci, ucj, ucij; } om_terms;

static om_terms om_elec(int ka, double ma, int kb, double mb, double r, double ci, double cj, double cij,
                        double kappa, double rc) {
  om_terms t = {0, 0, 0, 0, 0};
  const double ir = 1.0 / r;
  const double ir2 = ir * ir, ir3 = ir2 * ir, ir4 = ir3 * ir, ir5 = ir4 * ir;
  if (ka == OM_CHG && kb == OM_CHG) {
    t.u = ma * mb * ir;
    t.ur = -t.u * ir;
  } else if (ka == OM_CHG && kb == OM_DIP) {
    /* charge a in the potential of dipole b: q mu c_j / r^2 */
    const double p = ma * mb * ir2;
    t.u = p * cj;
    t.ur = -2.0 * t.u * ir;
    t.ucj = p;
  } else if (ka == OM_DIP && kb == OM_CHG) {
    /* dipole a in the field of charge b: -mu q c_i / r^2 */
    const double p = -ma * mb * ir2;
    t.u = p * ci;
    t.ur = -2.0 * t.u * ir;
    t.uci = p;
  } else if (ka == OM_CHG && kb == OM_QUAD) {
    const double p = ma * mb * ir3;
    t.u = p * (3.0 * cj * cj - 1.0) * 0.5;
    t.ur = -3.0 * t.u * ir;
    t.ucj = p * 3.0 * cj;
  } else if (ka == OM_QUAD && kb == OM_CHG) {
    const double p = ma * mb * ir3;
    t.u = p * (3.0 * ci * ci - 1.0) * 0.5;
    t.ur = -3.0 * t.u * ir;
    t.uci = p * 3.0 * ci;
  } else if (ka == OM_DIP && kb == OM_DIP) {
    const double p = ma * mb * ir3;
    t.u = p * (cij - 3.0 * ci * cj);
    t.ur = -3.0 * t.u * ir;
    t.uci = -3.0 * p * cj;
    t.ucj = -3.0 * p * ci;
    t.ucij = p;
    /* reaction field: -kappa mu_a mu_b (e_a.e_b) / r_c^3, no r dependence */
    const double prf = -kappa * ma * mb / (rc * rc * rc);
    t.u += prf * cij;
    t.ucij += prf;
  } else if (ka == OM_DIP && kb == OM_QUAD) {
    const double p = 1.5 * ma * mb * ir4;
    t.u = p * (ci - 5.0 * ci * cj * cj + 2.0 * cj * cij);
    t.ur = -4.0 * t.u * ir;
    t.uci = p * (1.0 - 5.0 * cj * cj);
    t.ucj = p * (-10.0 * ci * cj + 2.0 * cij);
    t.ucij = p * 2.0 * cj;
  } else if (ka == OM_QUAD && kb == OM_DIP) {
    const double p = -1.5 * ma * mb * ir4;
    t.u = p * (cj - 5.0 * cj * ci * ci + 2.0 * ci * cij);
    t.ur = -4.0 * t.u * ir;
    t.ucj = p * (1.0 - 5.0 * ci * ci);
    t.uci = p * (-10.0 * ci * cj + 2.0 * cij);
    t.ucij = p * 2.0 * ci;
  } else if (ka == OM_QUAD && kb == OM_QUAD) {
    const double p = 0.75 * ma * mb * ir5;
    const double s = cij - 5.0 * ci * cj;
    t.u = p * (1.0 - 5.0 * ci * ci - 5.0 * cj * cj - 15.0 * ci * ci * cj * cj + 2.0 * s * s);
    t.ur = -5.0 * t.u * ir;
    t.uci = p * (-10.0 * ci - 30.0 * ci * cj * cj - 20.0 * cj * s);
    t.ucj = p * (-10.0 * cj - 30.0 * cj * ci * ci - 20.0 * ci * s);
    t.ucij = p * 4.0 * s;
  }
  return t;
}

/* ---------------------------------------------------------------- per-molecule row sums */

typedef struct {
  double F[3], T[3], u, w, wd[3];
  int64_t nnb;
  double gsite[OM_MAXSITE][3]; /* dU/d(site position), world frame */
  double gaxis[OM_MAXSITE][3]; /* dU/d(site axis), world frame */
} om_row;

/* World-frame site offsets and axes of one molecule. */
static void om_sites_world(const om_model *m, int32_t comp, const double *q, double off[][3], double ax[][3]) {
  double A[3][3];
  if (q) {
    om_rotmat(q, A);
  } else {
    memset(A, 0, sizeof A);
    A[0][0] = A[1][1] = A[2][2] = 1.0;
  }
  for (int s = m->site_start[comp], a = 0; s < m->site_start[comp + 1]; ++s, ++a) {
    const double *rec = m->sites + (int64_t)s * OM_SITE_STRIDE;
    om_matvec(A, rec + 1, off[a]);
    om_matvec(A, rec + 4, ax[a]);
  }
}

/* All contributions of partner j to the row of molecule i (pair i-j counted from i's side). */
static void om_pair_into_row(const om_model *m, int64_t i, int64_t j, const double *pos, const double *quat,
                             const int32_t *comp, const double *box, double kappa, double rc2, om_row *row) {
  /* minimum image: choose the periodic image of j nearest to i, then separate */
  double dc[3];
  for (int k = 0; k < 3; ++k) {
    const double d0 = pos[3 * i + k] - pos[3 * j + k];
    const double s = nearbyint(d0 / box[k]);
    const double img = pos[3 * j + k] + s * box[k];
    dc[k] = pos[3 * i + k] - img;
  }
  const double r2 = fma(dc[2], dc[2], fma(dc[1], dc[1], dc[0] * dc[0]));
  if (!(r2 < rc2)) return;
  row->nnb += 1;

  const int32_t ci_ = comp[i], cj_ = comp[j];
  double offi[OM_MAXSITE][3], axi[OM_MAXSITE][3], offj[OM_MAXSITE][3], axj[OM_MAXSITE][3];
  om_sites_world(m, ci_, quat ? quat + 4 * i : NULL, offi, axi);
  om_sites_world(m, cj_, quat ? quat + 4 * j : NULL, offj, axj);
  const double xi_ = m->xi[ci_ * m->ncomp + cj_], eta_ = m->eta[ci_ * m->ncomp + cj_];

  double Fij[3] = {0, 0, 0};
  double uij = 0.0;
  const int na = m->site_start[ci_ + 1] - m->site_start[ci_];
  const int nb = m->site_start[cj_ + 1] - m->site_start[cj_];
  for (int a = 0; a < na; ++a) {
    const double *ra = m->sites + (int64_t)(m->site_start[ci_] + a) * OM_SITE_STRIDE;
    const int ka = (int)ra[0];
    for (int b = 0; b < nb; ++b) {
      const double *rb = m->sites + (int64_t)(m->site_start[cj_] + b) * OM_SITE_STRIDE;
      const int kb = (int)rb[0];
      if ((ka == OM_LJ) != (kb == OM_LJ)) continue; /* LJ sites meet LJ sites only */
      /* site separation: (r_i + o_a) - (image of r_j + o_b) */
      double R[3];
      for (int k = 0; k < 3; ++k) R[k] = (dc[k] + offi[a][k]) - offj[b][k];
      const double rr2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      double dUdR[3], ga[3] = {0, 0, 0};
      double u;
      if (ka == OM_LJ) {
        const double eps = xi_ * sqrt(ra[7] * rb[7]);
        const double sig = eta_ * 0.5 * (ra[8] + rb[8]);
        const double s2 = sig * sig / rr2;
        const double s6 = s2 * s2 * s2;
        u = 4.0 * eps * (s6 * s6 - s6);
        if (m->lj_shift) {
          const double c2 = sig * sig / rc2;
          const double c6 = c2 * c2 * c2;
          u -= 4.0 * eps * (c6 * c6 - c6);
        }
        /* du/dr * (1/r) = -24 eps (2 s^12 - s^6) / r^2 */
        const double durr = -24.0 * eps * (2.0 * s6 * s6 - s6) / rr2;
        for (int k = 0; k < 3; ++k) dUdR[k] = durr * R[k];
      } else {
        const double r = sqrt(rr2);
        double rh[3] = {R[0] / r, R[1] / r, R[2] / r};
        const double cia = (ka == OM_DIP || ka == OM_QUAD) ? om_dot(axi[a], rh) : 0.0;
        const double cjb = (kb == OM_DIP || kb == OM_QUAD) ? om_dot(axj[b], rh) : 0.0;
        const double cij = om_dot(axi[a], axj[b]);
        om_terms t = om_elec(ka, ra[7], kb, rb[7], r, cia, cjb, cij, kappa, m->rc);
        u = t.u;
        for (int k = 0; k < 3; ++k)
          dUdR[k] = t.ur * rh[k] + t.uci * (axi[a][k] - cia * rh[k]) / r + t.ucj * (axj[b][k] - cjb * rh[k]) / r;
        for (int k = 0; k < 3; ++k) ga[k] = t.uci * rh[k] + t.ucij * axj[b][k];
      }
      /* force on site a is -dU/dR; torque about i's COM: lever arm x force, minus axis x dU/de */
      double fa[3] = {-dUdR[0], -dUdR[1], -dUdR[2]};
      double lever[3], axt[3];
      om_cross(offi[a], fa, lever);
      om_cross(axi[a], ga, axt);
      for (int k = 0; k < 3; ++k) {
        Fij[k] += fa[k];
        row->T[k] += lever[k] - axt[k];
        row->gsite[a][k] += dUdR[k];
        row->gaxis[a][k] += ga[k];
      }
      uij += u;
    }
  }
  for (int k = 0; k < 3; ++k) {
    row->F[k] += Fij[k];
    row->wd[k] += 0.5 * dc[k] * Fij[k];
  }
  row->u += 0.5 * uij;
  row->w += 0.5 * (dc[0] * Fij[0] + dc[1] * Fij[1] + dc[2] * Fij[2]);
}

static double om_kappa(double eps_rf) {
  if (isinf(eps_rf)) return 1.0;
  return 2.0 * (eps_rf - 1.0) / (2.0 * eps_rf + 1.0);
}

/* Per-molecule sums over every partner j != i (rows = indices of the molecules wanted, or NULL
 * for all N).  Outputs are indexed by row position r = 0..nrows-1; any output may be NULL.
 * Positions are wrapped into the box first (same wrap as oracle_bin).
 *   F[r][3], T[r][3]: force and torque on molecule rows[r]
 *   u[r] = 1/2 sum_j u_ij, w[r] = 1/2 sum_j r_ij . F_ij, wd[r][3] = diagonal of the same tensor
 *   nnb[r] = number of partners with COM distance < r_c
 *   dquat[r][4] = dU/dq of molecule rows[r] through its site positions and axes.             */
int oracle_rows(const om_model *m, const double *pos_in, const double *quat, const int32_t *comp, int64_t N,
                const double *box, const int64_t *rows, int64_t nrows, double *F, double *T, double *u, double *w,
                double *wd, int64_t *nnb, double *dquat) {
  int32_t nc[3];
  if (!oracle_ncells(box, m->rc, nc)) return -1;
  for (int c = 0; c < m->ncomp; ++c)
    if (m->site_start[c + 1] - m->site_start[c] > OM_MAXSITE) return -2;
  double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  if (!pos) return -3;
  for (int64_t i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) pos[3 * i + k] = om_wrap(pos_in[3 * i + k], box[k]);
  const double kappa = om_kappa(m->eps_rf);
  const double rc2 = m->rc * m->rc;
  if (!rows) nrows = N;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows ? rows[r] : r;
    om_row row;
    memset(&row, 0, sizeof row);
    for (int64_t j = 0; j < N; ++j)
      if (j != i) om_pair_into_row(m, i, j, pos, quat, comp, box, kappa, rc2, &row);
    for (int k = 0; k < 3; ++k) {
      if (F) F[3 * r + k] = row.F[k];
      if (T) T[3 * r + k] = row.T[k];
      if (wd) wd[3 * r + k] = row.wd[k];
    }
    if (u) u[r] = row.u;
    if (w) w[r] = row.w;
    if (nnb) nnb[r] = row.nnb;
    if (dquat) {
      double dq[4] = {0, 0, 0, 0};
      if (quat) {
        const int32_t c = comp[i];
        for (int s = m->site_start[c], a = 0; s < m->site_start[c + 1]; ++s, ++a) {
          const double *rec = m->sites + (int64_t)s * OM_SITE_STRIDE;
          om_quat_grad(quat + 4 * i, rec + 1, row.gsite[a], dq);
          om_quat_grad(quat + 4 * i, rec + 4, row.gaxis[a], dq);
        }
      }
      for (int k = 0; k < 4; ++k) dquat[4 * r + k] = dq[k];
    }
  }
  free(pos);
  return 0;
}

/* Whole-system evaluation: every row, then the global sums in index order.
 * glob[5] = U, W, Wxx, Wyy, Wzz; *npairs = (sum_i nnb_i) / 2.                                 */
int oracle_all(const om_model *m, const double *pos, const double *quat, const int32_t *comp, int64_t N,
               const double *box, double *F, double *T, double *u, double *w, double *glob, int64_t *npairs) {
  double *uu = u ? u : (double *)malloc(sizeof(double) * (size_t)N);
  double *ww = w ? w : (double *)malloc(sizeof(double) * (size_t)N);
  double *wd = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  int64_t *nn = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
  int rcode = -3;
  if (uu && ww && wd && nn) {
    rcode = oracle_rows(m, pos, quat, comp, N, box, NULL, N, F, T, uu, ww, wd, nn, NULL);
    if (rcode == 0) {
      double U = 0, W = 0, Wd[3] = {0, 0, 0};
      int64_t np = 0;
      for (int64_t i = 0; i < N; ++i) {
        U += uu[i];
        W += ww[i];
        for (int k = 0; k < 3; ++k) Wd[k] += wd[3 * i + k];
        np += nn[i];
      }
      if (glob) {
        glob[0] = U;
        glob[1] = W;
        for (int k = 0; k < 3; ++k) glob[2 + k] = Wd[k];
      }
      if (npairs) *npairs = np / 2;
    }
  }
  if (!u) free(uu);
  if (!w) free(ww);
  free(wd);
  free(nn);
  return rcode;
}

/* ---------------------------------------------------------------- leapfrog (Sec. 3, Eqs. 2-5) */

static void om_qmul(const double *a, const double *b, double *out) {
  out[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  out[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  out[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  out[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

static void om_qnormalise(double *q) {
  const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= n;
}

/* Body-frame angular velocity from space-frame angular momentum: omega_b = I^-1 A(q)^T j,
 * with I_k^-1 taken as 0 where I_k = 0 (axis of a linear molecule).                          */
static void om_omega_body(const double *q, const double *j, const double *I, double *wb) {
  double A[3][3], jb[3];
  om_rotmat(q, A);
  om_matTvec(A, j, jb);
  for (int k = 0; k < 3; ++k) wb[k] = I[k] > 0.0 ? jb[k] / I[k] : 0.0;
}

/* q + h * (1/2) q' (x) (0, omega_b), where q' is the quaternion the rate is taken at. */
static void om_qadvance(const double *q, const double *qrate, const double *wb, double h, double *out) {
  double pw[4] = {0.0, wb[0], wb[1], wb[2]}, qd[4];
  om_qmul(qrate, pw, qd);
  for (int k = 0; k < 4; ++k) out[k] = q[k] + h * 0.5 * qd[k];
}

/* nsteps leapfrog steps.  State on entry: r(t), v(t - dt/2), q(t), j(t - dt/2) (space-frame
 * angular momentum).  Per step: forces and torques at t; v(t + dt/2) = v(t - dt/2) + dt F / m;
 * r(t + dt) = r(t) + dt v(t + dt/2), wrapped into the box.  Rotation (Fincham's leapfrog):
 * j(t) = j(t - dt/2) + dt/2 tau; q(t + dt/2) = q + dt/2 qdot(q, omega(t)), normalised;
 * j(t + dt/2) = j(t - dt/2) + dt tau; q(t + dt) = q + dt qdot(q(t + dt/2), omega(t + dt/2)),
 * normalised.  energies[s][4] = U(t), K_trans(t) with v(t) the mean of the two half-step
 * velocities, K_rot(t) = 1/2 sum_k jb_k(t)^2 / I_k over I_k > 0, W(t).
 * NVT (Sec. 2: the temperature is kept constant by velocity rescaling), when T_target > 0: after
 * each step the new half-step velocities and angular momenta are multiplied by
 * beta = sqrt(T_target / T(t)), T(t) = 2 (K_trans(t) + K_rot(t)) / f with k_B = 1 and
 * f = 3 N + the rotational degrees of freedom (the number of nonzero principal moments of each
 * rotating molecule); the energies row keeps K(t) before the rescaling.                      */
int oracle_step(const om_model *m, const double *mass, const double *inertia, double *pos, double *vel, double *quat,
                double *angmom, const int32_t *comp, int64_t N, const double *box, double dt, int64_t nsteps,
                double T_target, double *energies) {
  double *F = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *T = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  if (!F || !T) {
    free(F);
    free(T);
    return -3;
  }
  for (int64_t step = 0; step < nsteps; ++step) {
    double glob[5];
    int64_t np;
    int rcode = oracle_all(m, pos, quat, comp, N, box, F, T, NULL, NULL, glob, &np);
    if (rcode) {
      free(F);
      free(T);
      return rcode;
    }
    double Kt = 0.0, Kr = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      const int32_t c = comp[i];
      const double mi = mass[c];
      double kti = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double vold = vel[3 * i + k];
        const double vnew = vold + dt * F[3 * i + k] / mi;
        const double vmid = 0.5 * (vold + vnew);
        kti += vmid * vmid;
        vel[3 * i + k] = vnew;
        pos[3 * i + k] = om_wrap(pos[3 * i + k] + dt * vnew, box[k]);
      }
      Kt += 0.5 * mi * kti;
      const double *I = inertia + 3 * c;
      if (quat && angmom && (I[0] > 0.0 || I[1] > 0.0 || I[2] > 0.0)) {
        double *q = quat + 4 * i, *jm = angmom + 3 * i;
        const double *tq = T + 3 * i;
        double jt[3], wb[3], qh[4], jn[3], wbh[3], qn[4];
        for (int k = 0; k < 3; ++k) jt[k] = jm[k] + 0.5 * dt * tq[k];
        om_omega_body(q, jt, I, wb);
        for (int k = 0; k < 3; ++k) Kr += 0.5 * wb[k] * wb[k] * I[k];
        om_qadvance(q, q, wb, 0.5 * dt, qh);
        om_qnormalise(qh);
        for (int k = 0; k < 3; ++k) jn[k] = jm[k] + dt * tq[k];
        om_omega_body(qh, jn, I, wbh);
        om_qadvance(q, qh, wbh, dt, qn);
        om_qnormalise(qn);
        for (int k = 0; k < 4; ++k) q[k] = qn[k];
        for (int k = 0; k < 3; ++k) jm[k] = jn[k];
      }
    }
    if (energies) {
      energies[4 * step + 0] = glob[0];
      energies[4 * step + 1] = Kt;
      energies[4 * step + 2] = Kr;
      energies[4 * step + 3] = glob[1];
    }
    if (T_target > 0.0) {
      double f = 3.0 * (double)N;
      for (int64_t i = 0; i < N; ++i) {
        const double *I = inertia + 3 * comp[i];
        if (quat && angmom) f += (I[0] > 0.0) + (I[1] > 0.0) + (I[2] > 0.0);
      }
      const double K = Kt + Kr;
      const double beta = K > 0.0 ? sqrt(0.5 * f * T_target / K) : 1.0;
      for (int64_t i = 0; i < N; ++i) {
        for (int k = 0; k < 3; ++k) vel[3 * i + k] *= beta;
        const double *I = inertia + 3 * comp[i];
        if (quat && angmom && (I[0] > 0.0 || I[1] > 0.0 || I[2] > 0.0))
          for (int k = 0; k < 3; ++k) angmom[3 * i + k] *= beta;
      }
    }
  }
  free(F);
  free(T);
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
