// libmdcell host side: argument validation, model tables, buffer management, launch sequencing,
// error codes, device status word and event-based kernel timing.  Every compute step runs in the
// HIP kernels of md_cells.hip, md_pair.hip, md_step.hip and md_adjoint.hip.

#include <cmath>
#include <cstring>
#include <string>

#include "md_internal.h"

using namespace mdcell;

namespace mdcell {

static thread_local std::string g_err;

int set_error(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return MD_OK;
  return set_error(MD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device allocation: MD_ENOMEM when the device is out of memory, MD_EHIP for other failures.
static int dalloc(void **p, size_t bytes, const char *what) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(e == hipErrorOutOfMemory ? MD_ENOMEM : MD_EHIP,
                     std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
  }
  return MD_OK;
}

template <typename T> static void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

// Grow a device buffer to hold at least n elements of T (contents not preserved).
template <typename T> static int grow(T *&p, int64_t &cap, int64_t n, const char *what) {
  if (n <= cap && p) return MD_OK;
  dfree(p);
  cap = 0;
  int rc = dalloc((void **)&p, sizeof(T) * (size_t)(n > 0 ? n : 1), what);
  if (rc) return rc;
  cap = n;
  return MD_OK;
}

void prof_begin(md_model *m, int group, hipStream_t s, hipEvent_t *a) {
  *a = nullptr;
  if (!m->profiling) return;
  if (hipEventCreate(a) != hipSuccess) {
    *a = nullptr;
    return;
  }
  (void)hipEventRecord(*a, s);
  (void)group;
}

void prof_end(md_model *m, int group, hipStream_t s, hipEvent_t a) {
  if (!m->profiling || !a) return;
  hipEvent_t b;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  (void)hipEventRecord(b, s);
  m->events.push_back({group, a, b});
}

// Cells per axis: floor(L / r_c), reduced until the cell edge exceeds r_c by a relative margin of
// 2^-30 (so rounding of a bin index can never hide a partner inside the cutoff).
static bool cells_per_axis(const double *box, double rc, int32_t nc[3]) {
  for (int k = 0; k < 3; ++k) {
    double n = std::floor(box[k] / rc);
    while (n >= 1.0 && box[k] / n < rc * (1.0 + 0x1p-30)) n -= 1.0;
    if (n < 3.0 || n > 1.0e6) return false;
    nc[k] = (int32_t)n;
  }
  return true;
}

static int finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static int sync_check(md_model *m, hipStream_t s) {
  if (!(m->flags & MD_CHECK)) return MD_OK;
  int rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc) return rc;
  int32_t st = 0;
  rc = check_hip(hipMemcpy(&st, m->status, sizeof st, hipMemcpyDeviceToHost), "hipMemcpy(status)");
  if (rc) return rc;
  if (st) {
    launch_fill_i32(m->status, 1, 0, s);
    (void)hipStreamSynchronize(s);
    return set_error(MD_EDEVICE, "device status word " + std::to_string(st) +
                                     " (1: non-finite position, 2: component id, 4: non-unit quaternion, "
                                     "16: fix-up list full)");
  }
  return MD_OK;
}

// Lorentz-Berthelot mixing per LJ site pair (Sec. 2), with the optional LJTS shift u_ab(r_c) and
// the adjoint's per-pair factors; recomputed whenever the site parameters change.
static void mix_lj(ModelDev &h) {
  std::memset(h.lj, 0, sizeof h.lj);
  std::memset(h.shift_sum, 0, sizeof h.shift_sum);
  const int ncomp = h.ncomp;
  for (int A = 0; A < ncomp; ++A)
    for (int B = 0; B < ncomp; ++B)
      for (int a = 0; a < h.comp[A].n_lj; ++a)
        for (int b = 0; b < h.comp[B].n_lj; ++b) {
          const double eps = h.xi[A][B] * std::sqrt(h.comp[A].lj_eps[a] * h.comp[B].lj_eps[b]);
          const double sig = h.eta[A][B] * 0.5 * (h.comp[A].lj_sig[a] + h.comp[B].lj_sig[b]);
          LJPair &p = h.lj[A][B][a][b];
          p.eps4 = 4.0 * eps;
          p.eps24 = 24.0 * eps;
          p.sig2 = sig * sig;
          p.pe = 0.5 / h.comp[A].lj_eps[a];
          p.ps = 0.5 * h.eta[A][B] * 4.0 * eps / sig;
          if (h.lj_shift) {
            const double c2 = sig * sig / h.rc2;
            const double c6 = c2 * c2 * c2;
            p.shift = 4.0 * eps * (c6 * c6 - c6);
            p.csh = 12.0 * c6 * c6 - 6.0 * c6;
          } else {
            p.shift = 0.0;
            p.csh = 0.0;
          }
          h.shift_sum[A][B] += p.shift;
        }
}

// Walk the parameter vector in the md_param_count layout; f(value reference, is_lj_magnitude)
template <typename F> void for_each_param(ModelDev &h, F f) {
  for (int c = 0; c < h.ncomp; ++c) {
    CompDev &cd = h.comp[c];
    for (int a = 0; a < cd.n_lj; ++a) {
      f(cd.lj_eps[a], true), f(cd.lj_sig[a], true);
      for (int k = 0; k < 3; ++k) f(cd.lj_pos[a][k], false);
    }
    for (int a = 0; a < cd.n_chg; ++a) {
      f(cd.chg_q[a], false);
      for (int k = 0; k < 3; ++k) f(cd.chg_pos[a][k], false);
    }
    for (int a = 0; a < cd.n_dip; ++a) {
      f(cd.dip_mu[a], false);
      for (int k = 0; k < 3; ++k) f(cd.dip_pos[a][k], false);
    }
    for (int a = 0; a < cd.n_quad; ++a) {
      f(cd.quad_Q[a], false);
      for (int k = 0; k < 3; ++k) f(cd.quad_pos[a][k], false);
    }
  }
}

}  // namespace mdcell

extern "C" {

const char *md_last_error(void) { return g_err.c_str(); }

int md_model_create(const md_component_desc *comps, int32_t ncomp, const double *xi, const double *eta, double rc,
                    double eps_rf, uint32_t flags, md_model **out) {
  if (!out) return set_error(MD_EINVAL, "md_model_create: out is NULL");
  *out = nullptr;
  if (!comps) return set_error(MD_EINVAL, "md_model_create: comps is NULL");
  if (ncomp < 1) return set_error(MD_EINVAL, "md_model_create: ncomp < 1");
  if (ncomp > MD_MAX_COMP) return set_error(MD_ECOMP, "md_model_create: ncomp exceeds MD_MAX_COMP");
  if (!std::isfinite(rc)) return set_error(MD_ENONFINITE, "md_model_create: r_c not finite");
  if (!(rc > 0.0)) return set_error(MD_EINVAL, "md_model_create: r_c <= 0");
  if (std::isnan(eps_rf) || !(eps_rf > 0.0)) return set_error(MD_EINVAL, "md_model_create: eps_rf must be > 0");
  if (flags & ~(MD_LJ_SHIFT | MD_CHECK | MD_HALF_SHELL | MD_SUBCELLS))
    return set_error(MD_EINVAL, "md_model_create: unknown flag");
  md_model tmp;
  ModelDev &h = tmp.host;
  std::memset(&h, 0, sizeof h);
  h.ncomp = ncomp;
  h.lj_shift = (flags & MD_LJ_SHIFT) ? 1 : 0;
  h.rc = rc;
  h.rc2 = rc * rc;
  h.kappa = std::isinf(eps_rf) ? 1.0 : 2.0 * (eps_rf - 1.0) / (2.0 * eps_rf + 1.0);
  h.kappa_rc3 = h.kappa / (rc * rc * rc);
  Shape mx{0, 0, 0, 0};
  for (int c = 0; c < ncomp; ++c) {
    const md_component_desc &d = comps[c];
    CompDev &cd = h.comp[c];
    if (d.n_lj < 0 || d.n_chg < 0 || d.n_dip < 0 || d.n_quad < 0)
      return set_error(MD_EINVAL, "md_model_create: negative site count");
    if (d.n_lj > MD_MAX_LJ || d.n_chg > MD_MAX_CHG || d.n_dip > MD_MAX_DIP || d.n_quad > MD_MAX_QUAD)
      return set_error(MD_ECOMP, "md_model_create: site count exceeds the compiled limits");
    if (d.n_lj + d.n_chg + d.n_dip + d.n_quad == 0) return set_error(MD_EINVAL, "md_model_create: component without sites");
    if ((d.n_lj && (!d.lj_pos || !d.lj_eps || !d.lj_sigma)) || (d.n_chg && (!d.chg_pos || !d.chg_q)) ||
        (d.n_dip && (!d.dip_pos || !d.dip_dir || !d.dip_mu)) || (d.n_quad && (!d.quad_pos || !d.quad_dir || !d.quad_Q)))
      return set_error(MD_EINVAL, "md_model_create: NULL site table");
    if (!finite_pos(d.mass)) return set_error(MD_EINVAL, "md_model_create: mass must be finite and > 0");
    cd.n_lj = d.n_lj, cd.n_chg = d.n_chg, cd.n_dip = d.n_dip, cd.n_quad = d.n_quad;
    cd.mass = d.mass;
    cd.inv_mass = 1.0 / d.mass;
    cd.rotates = 0;
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(d.inertia[k]) || d.inertia[k] < 0.0)
        return set_error(MD_EINVAL, "md_model_create: inertia must be finite and >= 0");
      cd.inertia[k] = d.inertia[k];
      cd.inv_inertia[k] = d.inertia[k] > 0.0 ? 1.0 / d.inertia[k] : 0.0;
      if (d.inertia[k] > 0.0) cd.rotates = 1;
    }
    auto fin3 = [](const double *p, int n) {
      for (int i = 0; i < 3 * n; ++i)
        if (!std::isfinite(p[i])) return false;
      return true;
    };
    auto fin1 = [](const double *p, int n) {
      for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
      return true;
    };
    if ((d.n_lj && (!fin3(d.lj_pos, d.n_lj) || !fin1(d.lj_eps, d.n_lj) || !fin1(d.lj_sigma, d.n_lj))) ||
        (d.n_chg && (!fin3(d.chg_pos, d.n_chg) || !fin1(d.chg_q, d.n_chg))) ||
        (d.n_dip && (!fin3(d.dip_pos, d.n_dip) || !fin3(d.dip_dir, d.n_dip) || !fin1(d.dip_mu, d.n_dip))) ||
        (d.n_quad && (!fin3(d.quad_pos, d.n_quad) || !fin3(d.quad_dir, d.n_quad) || !fin1(d.quad_Q, d.n_quad))))
      return set_error(MD_ENONFINITE, "md_model_create: non-finite site table entry");
    for (int a = 0; a < d.n_lj; ++a) {
      if (!(d.lj_eps[a] > 0.0) || !(d.lj_sigma[a] > 0.0))
        return set_error(MD_EINVAL, "md_model_create: LJ epsilon and sigma must be > 0");
      for (int k = 0; k < 3; ++k) cd.lj_pos[a][k] = d.lj_pos[3 * a + k];
      cd.lj_eps[a] = d.lj_eps[a];
      cd.lj_sig[a] = d.lj_sigma[a];
    }
    for (int a = 0; a < d.n_chg; ++a) {
      for (int k = 0; k < 3; ++k) cd.chg_pos[a][k] = d.chg_pos[3 * a + k];
      cd.chg_q[a] = d.chg_q[a];
    }
    for (int a = 0; a < d.n_dip; ++a) {
      for (int k = 0; k < 3; ++k) cd.dip_pos[a][k] = d.dip_pos[3 * a + k], cd.dip_dir[a][k] = d.dip_dir[3 * a + k];
      cd.dip_mu[a] = d.dip_mu[a];
    }
    for (int a = 0; a < d.n_quad; ++a) {
      for (int k = 0; k < 3; ++k) cd.quad_pos[a][k] = d.quad_pos[3 * a + k], cd.quad_dir[a][k] = d.quad_dir[3 * a + k];
      cd.quad_Q[a] = d.quad_Q[a];
    }
    mx.lj = std::max(mx.lj, (int)d.n_lj), mx.chg = std::max(mx.chg, (int)d.n_chg);
    mx.dip = std::max(mx.dip, (int)d.n_dip), mx.quad = std::max(mx.quad, (int)d.n_quad);
  }
  for (int a = 0; a < ncomp; ++a)
    for (int b = 0; b < ncomp; ++b) {
      const double x = xi ? xi[a * ncomp + b] : 1.0, e = eta ? eta[a * ncomp + b] : 1.0;
      if (!std::isfinite(x) || !std::isfinite(e)) return set_error(MD_ENONFINITE, "md_model_create: xi/eta not finite");
      if (!(x > 0.0) || !(e > 0.0)) return set_error(MD_EINVAL, "md_model_create: xi/eta must be > 0");
      h.xi[a][b] = x, h.eta[a][b] = e;
    }
  mix_lj(h);
  const md_component_desc &d0 = comps[0];
  tmp.single_site = ncomp == 1 && d0.n_lj == 1 && d0.n_chg + d0.n_dip + d0.n_quad == 0 && d0.lj_pos[0] == 0.0 &&
                    d0.lj_pos[1] == 0.0 && d0.lj_pos[2] == 0.0;
  const bool is2q = mx.lj == 2 && mx.chg == 0 && mx.dip == 0 && mx.quad == 1;
  const bool is3d = mx.lj == 3 && mx.chg == 0 && mx.dip == 1 && mx.quad == 0;
  tmp.fixed_shape = ncomp == 1 && (is2q || is3d);
  if (tmp.single_site) tmp.shape = Shape{1, 0, 0, 0};
  else if (tmp.fixed_shape) tmp.shape = mx;
  else tmp.shape = Shape{MD_MAX_LJ, MD_MAX_CHG, MD_MAX_DIP, MD_MAX_QUAD};
  h.sl = tmp.shape.lj, h.sc = tmp.shape.chg, h.sd = tmp.shape.dip, h.sq = tmp.shape.quad;
  // parameter-gradient layout
  int64_t off = 0;
  for (int c = 0; c < ncomp; ++c) {
    tmp.param_off.push_back(off);
    off += 5 * comps[c].n_lj + 4 * (comps[c].n_chg + comps[c].n_dip + comps[c].n_quad);
  }
  tmp.nparam = off;
  for (int c = 0; c < ncomp; ++c) h.param_off[c] = (int32_t)tmp.param_off[c];
  h.nparam = (int32_t)off;
  tmp.flags = flags;

  md_model *m = new md_model(tmp);
  int rcode = MD_OK;
  if ((rcode = dalloc((void **)&m->dev, sizeof(ModelDev), "model")) ||
      (rcode = check_hip(hipMemcpy(m->dev, &m->host, sizeof(ModelDev), hipMemcpyHostToDevice), "hipMemcpy(model)")) ||
      (rcode = dalloc((void **)&m->status, sizeof(int32_t), "status")) ||
      (rcode = check_hip(hipMemset(m->status, 0, sizeof(int32_t)), "hipMemset(status)")) ||
      (rcode = dalloc((void **)&m->red2, sizeof(double) * 256 * 256, "reduction")) ||
      (rcode = dalloc((void **)&m->uw, sizeof(double) * 64, "sums")) ||
      (rcode = dalloc((void **)&m->bad, sizeof(unsigned long long) * (1 + BAD_CAP), "fix-up list")) ||
      (rcode = check_hip(hipMemset(m->bad, 0, sizeof(unsigned long long)), "hipMemset(fix-up list)"))) {
    md_model_destroy(m);
    return rcode;
  }
  *out = m;
  return MD_OK;
}

int md_model_destroy(md_model *m) {
  if (!m) return MD_OK;
  for (auto &e : m->events) (void)hipEventDestroy(e.a), (void)hipEventDestroy(e.b);
  if (m->side) {
    (void)hipStreamSynchronize(m->side);
    (void)hipStreamDestroy(m->side);
  }
  for (int k = 0; k < 2; ++k) {
    if (m->ev_leap[k]) (void)hipEventDestroy(m->ev_leap[k]);
    if (m->ev_red[k]) (void)hipEventDestroy(m->ev_red[k]);
  }
  dfree(m->dev);
  dfree(m->status);
  dfree(m->partial);
  dfree(m->rows);
  dfree(m->bad);
  dfree(m->red2);
  dfree(m->pgrad);
  dfree(m->force);
  dfree(m->torque);
  dfree(m->uw);
  delete m;
  return MD_OK;
}

int64_t md_param_count(const md_model *m) { return m ? m->nparam : -1; }

int md_model_get_params(const md_model *m, double *params) {
  if (!m || !params) return set_error(MD_EINVAL, "md_model_get_params: NULL argument");
  ModelDev h = m->host;
  int64_t k = 0;
  for_each_param(h, [&](double &v, bool) { params[k++] = v; });
  return MD_OK;
}

int md_model_set_params(md_model *m, const double *params) {
  if (!m || !params) return set_error(MD_EINVAL, "md_model_set_params: NULL argument");
  for (int64_t k = 0; k < m->nparam; ++k)
    if (!std::isfinite(params[k])) return set_error(MD_ENONFINITE, "md_model_set_params: non-finite parameter");
  ModelDev h = m->host;
  int64_t k = 0;
  bool ok = true;
  for_each_param(h, [&](double &v, bool positive) {
    v = params[k++];
    if (positive && !(v > 0.0)) ok = false;
  });
  if (!ok) return set_error(MD_EINVAL, "md_model_set_params: LJ epsilon and sigma must be > 0");
  if (m->single_site && (h.comp[0].lj_pos[0][0] != 0.0 || h.comp[0].lj_pos[0][1] != 0.0 || h.comp[0].lj_pos[0][2] != 0.0))
    return set_error(MD_EINVAL, "md_model_set_params: the site of a single-site model stays at the centre of mass");
  mix_lj(h);
  // kernels still reading the old tables finish first
  int rc = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if (rc) return rc;
  if ((rc = check_hip(hipMemcpy(m->dev, &h, sizeof(ModelDev), hipMemcpyHostToDevice), "hipMemcpy(model)"))) return rc;
  m->host = h;
  return MD_OK;
}

int md_cells_create(md_cells **out) {
  if (!out) return set_error(MD_EINVAL, "md_cells_create: out is NULL");
  *out = new md_cells();
  return MD_OK;
}

int md_cells_destroy(md_cells *c) {
  if (!c) return MD_OK;
  dfree(c->cell_of), dfree(c->cellv), dfree(c->slot), dfree(c->tmp), dfree(c->perm), dfree(c->perm_prev);
  dfree(c->scomp);
  dfree(c->count), dfree(c->start), dfree(c->bsum), dfree(c->lstart), dfree(c->cstart);
  dfree(c->sx), dfree(c->sy), dfree(c->sz), dfree(c->svec), dfree(c->squat);
  delete c;
  return MD_OK;
}

int md_cells_view(const md_cells *c, md_cells_info *out) {
  if (!c || !out) return set_error(MD_EINVAL, "md_cells_view: NULL argument");
  if (!c->built) return set_error(MD_EINVAL, "md_cells_view: cells not built");
  if (!c->cell_of_valid) {  // the caller-order cell ids, formed once per build on request
    md_cells *cm = const_cast<md_cells *>(c);
    const hipStream_t s = c->model ? c->model->last_stream : nullptr;
    int rc = launch_cell_of(c, s);
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (rc) return rc;
    cm->cell_of_valid = true;
  }
  out->N = c->N;
  out->ncell = c->ncell;
  for (int k = 0; k < 3; ++k) out->nc[k] = c->nc[k], out->box[k] = c->box[k];
  out->cell_of = c->cell_of;
  out->cell_start = c->sub ? c->cstart : c->start;
  out->perm = c->perm;
  out->sub_start = c->sub ? c->start : nullptr;
  return MD_OK;
}

int md_build_cells(md_model *m, md_cells *c, const double *pos, const double *quat, const int32_t *comp, int64_t N,
                   const double box[3], void *stream) {
  if (!m || !c || !pos || !box) return set_error(MD_EINVAL, "md_build_cells: NULL argument");
  if (N <= 0 || N >= (int64_t)1 << 31) return set_error(MD_EINVAL, "md_build_cells: N must be in [1, 2^31)");
  if (!m->single_site && !quat) return set_error(MD_EINVAL, "md_build_cells: multi-site model needs quaternions");
  if (m->host.ncomp > 1 && !comp) return set_error(MD_EINVAL, "md_build_cells: mixture needs component ids");
  for (int k = 0; k < 3; ++k) {
    if (!std::isfinite(box[k])) return set_error(MD_ENONFINITE, "md_build_cells: box not finite");
    if (!(box[k] > 0.0)) return set_error(MD_EINVAL, "md_build_cells: box <= 0");
  }
  int32_t nc[3];
  if (!cells_per_axis(box, m->host.rc, nc))
    return set_error(MD_EBOX, "md_build_cells: a box side holds fewer than 3 cells of edge > r_c");
  const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  if (ncell >= ((int64_t)1 << 31) - 8) return set_error(MD_EBOX, "md_build_cells: too many cells");
  hipStream_t s = (hipStream_t)stream;
  m->last_stream = s;
  const int nvec = m->single_site ? 0 : m->shape.nvec();
  int rc;
  int64_t capN = c->cap_N, capC = c->cap_cell, capB = c->cap_blocks;
  // a rebuild of the same N visits the molecules in the previous sorted order (fewer contended
  // atomics, near-sequential writes); the result does not depend on the visiting order
  const bool reuse_order = c->built && c->N == N && N <= capN;
  if (N > capN) {
    int64_t cap = 0;
    if ((rc = grow(c->cell_of, cap, N, "cell_of")) || (cap = 0, rc = grow(c->cellv, cap, N, "cellv")) ||
        (cap = 0, rc = grow(c->slot, cap, N, "slot")) ||
        (cap = 0, rc = grow(c->tmp, cap, N, "tmp")) || (cap = 0, rc = grow(c->perm, cap, N, "perm")) ||
        (cap = 0, rc = grow(c->perm_prev, cap, N, "perm")) ||
        (cap = 0, rc = grow(c->scomp, cap, N, "scomp")) || (cap = 0, rc = grow(c->sx, cap, N, "sx")) ||
        (cap = 0, rc = grow(c->sy, cap, N, "sy")) || (cap = 0, rc = grow(c->sz, cap, N, "sz"))) {
      c->cap_N = 0;
      return rc;
    }
    c->cap_N = N;
    c->cap_nvec = 0;
  }
  if ((int64_t)nvec * N > (int64_t)c->cap_nvec * c->cap_N || !c->svec) {
    int64_t cap = 0;
    if ((rc = grow(c->svec, cap, std::max<int64_t>(1, (int64_t)nvec * 3 * c->cap_N), "svec"))) return rc;
    c->cap_nvec = nvec;
  }
  if (!m->single_site && (rc = grow(c->squat, c->cap_squat, 4 * N, "squat"))) return rc;
  // half-edge cells: single-site models evaluated from both ends, on request
  const bool sub = (m->flags & MD_SUBCELLS) && m->single_site && !(m->flags & MD_HALF_SHELL);
  const int64_t nbin = sub ? 8 * ncell : ncell;
  if (nbin + 1 > capC) {
    int64_t cap = 0;
    c->counts_zero = false;
    c->cap_cell = 0;  // stays 0 if an allocation below fails, so the next build retries
    if ((rc = grow(c->count, cap, nbin + 1, "count")) || (cap = 0, rc = grow(c->start, cap, nbin + 1, "start")) ||
        (cap = 0, rc = grow(c->lstart, cap, nbin + 1, "lstart")))
      return rc;
    c->cap_cell = nbin + 1;
  }
  if (sub && (rc = grow(c->cstart, c->cap_cstart, ncell + 1, "cstart"))) return rc;
  const int64_t nb = (nbin + 1023) / 1024 + 1;
  if (nb > capB) {
    int64_t cap = 0;
    c->cap_blocks = 0;
    if ((rc = grow(c->bsum, cap, nb, "bsum"))) return rc;
    c->cap_blocks = nb;
  }
  c->N = N;
  c->ncell = ncell;
  c->sub = sub;
  for (int k = 0; k < 3; ++k) c->nc[k] = nc[k], c->box[k] = box[k];
  c->nvec = nvec;
  c->model = m;
  c->built = false;
  const double inv_h[3] = {(double)nc[0] / box[0], (double)nc[1] / box[1], (double)nc[2] / box[2]};
  const double inv_hh[3] = {(double)(2 * nc[0]) / box[0], (double)(2 * nc[1]) / box[1], (double)(2 * nc[2]) / box[2]};
  hipEvent_t ev;
  prof_begin(m, PROF_BUILD, s, &ev);
  const int32_t *order = nullptr;
  if (reuse_order) {
    std::swap(c->perm, c->perm_prev);
    order = c->perm_prev;
  }
  rc = launch_build(m, c, pos, quat, m->host.ncomp > 1 ? comp : nullptr, N, inv_h, inv_hh, order, s);
  prof_end(m, PROF_BUILD, s, ev);
  if (rc) return rc;
  c->order = order;
  c->cell_of_valid = false;
  c->built = true;
  return sync_check(m, s);
}

// Scratch of one pair evaluation, in doubles: the block partials, and for the half-shell kernels
// (multi-site models, MD_HALF_SHELL) the per-molecule partner rows of force (and torque) in the
// path's precision followed, 256-byte aligned, by the FP64 u, w and count rows when per-molecule
// outputs are wanted (nq = 9).
struct PairScratch {
  int64_t partial, ft, uw;  // doubles of each part; rows = ft + uw
};
static PairScratch pair_scratch(const md_model *m, const md_cells *c, int precision, int nq) {
  PairScratch r{};
  r.partial = pair_blocks(c->ncell) * PARTIAL_COLS + KIN_COLS * ((3 * c->N + 255) / 256 + (c->N + 255) / 256);
  const bool half_shell = !m->single_site || (m->flags & MD_HALF_SHELL);
  if (half_shell) {
    const int64_t ft_bytes = (int64_t)N3_ROWS * c->N * (m->single_site ? 3 : 6) * (precision == MD_FP32 ? 4 : 8);
    r.ft = (ft_bytes + 255) / 256 * 32;
    r.uw = nq > 6 ? (int64_t)N3_ROWS * c->N * 3 : 0;
  }
  return r;
}

// Pair kernel (+ the reduction of its block partials unless reduce is false: md_step reduces them
// together with the leapfrog's kinetic-energy partials, which follow them in m->partial).  With
// scratch given (md_forces_noalloc) the partials and rows live there and nothing is allocated.
static int forces_impl(md_model *m, const md_cells *c, int precision, double *force, double *torque, double *u_mol,
                       double *w_mol, int32_t *nnb_mol, double *uw, int64_t *npairs, double *erow, hipStream_t s,
                       bool reduce = true, int64_t *nblocks_out = nullptr, double *partial = nullptr,
                       double *scratch = nullptr) {
  const int nq = (u_mol || w_mol || nnb_mol) ? 9 : 6;
  const PairScratch need = pair_scratch(m, c, precision, nq);
  int rc;
  double *rows = nullptr;
  if (scratch) {
    partial = scratch;
    rows = scratch + (need.partial + 31) / 32 * 32;
  } else {
    if ((rc = grow(m->partial, m->cap_partial, need.partial, "partial"))) return rc;
    if (need.ft && (rc = grow(m->rows, m->cap_rows, need.ft + need.uw, "pair rows"))) return rc;
    rows = m->rows;
    if (!partial) partial = m->partial;
  }
  PairOut o{force, torque, u_mol, w_mol, nnb_mol, partial, rows, rows ? rows + need.ft : nullptr, c->N, nq, m->status,
            m->bad};
  int64_t nblocks = 0;
  hipEvent_t ev;
  if (!scratch) prof_begin(m, PROF_PAIR, s, &ev);
  rc = launch_pair(m, c, precision, o, s, &nblocks);
  if (!scratch) prof_end(m, PROF_PAIR, s, ev);
  if (rc) return rc;
  if (nblocks_out) *nblocks_out = nblocks;
  return reduce ? launch_reduce_forces(m, nblocks, partial, uw, npairs, erow, s) : MD_OK;
}

int md_forces(md_model *m, const md_cells *c, int precision, double *force, double *torque, double *u_mol,
              double *w_mol, int32_t *nnb_mol, double *uw, int64_t *npairs, void *stream) {
  if (!m || !c || !force || !uw) return set_error(MD_EINVAL, "md_forces: NULL argument");
  if (precision != MD_FP64 && precision != MD_FP32) return set_error(MD_EINVAL, "md_forces: bad precision");
  if (!c->built || c->model != m) return set_error(MD_EINVAL, "md_forces: cells not built with this model");
  hipStream_t s = (hipStream_t)stream;
  m->last_stream = s;
  int rc = forces_impl(m, c, precision, force, torque, u_mol, w_mol, nnb_mol, uw, npairs, nullptr, s);
  if (rc) return rc;
  return sync_check(m, s);
}

int md_forces_noalloc(md_model *m, const md_cells *c, int precision, double *force, double *torque, double *u_mol,
                      double *w_mol, int32_t *nnb_mol, double *uw, int64_t *npairs, void *stream) {
  if (!m || !c || !force || !uw) return set_error(MD_EINVAL, "md_forces_noalloc: NULL argument");
  if (precision != MD_FP64 && precision != MD_FP32) return set_error(MD_EINVAL, "md_forces_noalloc: bad precision");
  if (!c->built || c->model != m) return set_error(MD_EINVAL, "md_forces_noalloc: cells not built with this model");
  const int nq = (u_mol || w_mol || nnb_mol) ? 9 : 6;
  const PairScratch need = pair_scratch(m, c, precision, nq);
  const int64_t bytes = 8 * ((need.partial + 31) / 32 * 32 + need.ft + need.uw);
  if (bytes > (int64_t)MD_NOALLOC_SCRATCH_BYTES)
    return set_error(MD_EINVAL, "md_forces_noalloc: this configuration needs " + std::to_string(bytes) +
                                    " bytes of scratch, the static array holds " +
                                    std::to_string((int64_t)MD_NOALLOC_SCRATCH_BYTES));
  void *scratch = nullptr;
  int rc = noalloc_scratch(&scratch);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  m->last_stream = s;
  rc = forces_impl(m, c, precision, force, torque, u_mol, w_mol, nnb_mol, uw, npairs, nullptr, s, true, nullptr,
                   nullptr, (double *)scratch);
  if (rc) return rc;
  return sync_check(m, s);
}

int md_step(md_model *m, md_cells *c, double *pos, double *vel, double *quat, double *angmom, const int32_t *comp,
            int64_t N, const double box[3], double dt, int64_t nsteps, int precision, double *energies, void *stream) {
  if (!m || !c || !pos || !vel || !box) return set_error(MD_EINVAL, "md_step: NULL argument");
  if (precision != MD_FP64 && precision != MD_FP32) return set_error(MD_EINVAL, "md_step: bad precision");
  if (!std::isfinite(dt)) return set_error(MD_ENONFINITE, "md_step: dt not finite");
  if (!(dt > 0.0)) return set_error(MD_EINVAL, "md_step: dt <= 0");
  if (nsteps < 0) return set_error(MD_EINVAL, "md_step: nsteps < 0");
  if (!m->single_site && (!quat || !angmom)) return set_error(MD_EINVAL, "md_step: multi-site model needs quat and angmom");
  hipStream_t s = (hipStream_t)stream;
  m->last_stream = s;
  int rc;
  if (N > m->cap_step) {
    int64_t cap = 0;
    if ((rc = grow(m->force, cap, 3 * N, "step force")) || (cap = 0, rc = grow(m->torque, cap, 3 * N, "step torque")))
      return rc;
    m->cap_step = N;
  }
  const bool nvt = m->T_target > 0.0;
  // with an energies row or the thermostat, each step's reduction (and the thermostat's velocity
  // rescaling) goes to the side stream and overlaps the next step's build and forces, which do
  // not read the velocities; the next leapfrog waits for it.  The pair and kinetic partial rows
  // then alternate between two slots
  const bool overlap = (energies || nvt) && nsteps > 1;
  int64_t slot_sz = 0;
  // an error return after a side-stream reduction has been queued first orders the caller's
  // stream after the last one, so that no queued reduction writes `energies` after the return
  int last_red = -1;
  auto fail = [&](int code) {
    if (last_red >= 0) (void)hipStreamWaitEvent(s, m->ev_red[last_red], 0);
    return code;
  };
  for (int64_t st = 0; st < nsteps; ++st) {
    if ((rc = md_build_cells(m, c, pos, quat, comp, N, box, stream))) return fail(rc);
    if (overlap && st == 0) {  // the grid is fixed within the call (same box, same cutoff)
      slot_sz = pair_blocks(c->ncell) * PARTIAL_COLS + KIN_COLS * ((3 * N + 255) / 256 + (N + 255) / 256);
      if ((rc = grow(m->partial, m->cap_partial, 2 * slot_sz, "partial"))) return rc;
      if (!m->side && (rc = check_hip(hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking), "hipStreamCreate")))
        return rc;
      for (int k = 0; k < 2; ++k)
        if ((!m->ev_leap[k] && (rc = check_hip(hipEventCreateWithFlags(&m->ev_leap[k], hipEventDisableTiming), "hipEventCreate"))) ||
            (!m->ev_red[k] && (rc = check_hip(hipEventCreateWithFlags(&m->ev_red[k], hipEventDisableTiming), "hipEventCreate"))))
          return rc;
    }
    const int slot = (int)(st & 1);
    // partial rows: the slot of this step, or (without overlap) the buffer forces_impl sizes,
    // read back after the call, which may allocate it
    double *part = overlap ? m->partial + slot * slot_sz : nullptr;
    // the reduction of step st - 2 has read this slot
    if (overlap && st >= 2 && (rc = check_hip(hipStreamWaitEvent(s, m->ev_red[slot], 0), "hipStreamWaitEvent")))
      return fail(rc);
    double *erow = energies ? energies + 4 * st : nullptr;
    int64_t nbp = 0;
    if ((rc = forces_impl(m, c, precision, m->force, m->single_site ? nullptr : m->torque, nullptr, nullptr, nullptr,
                          m->uw + 8, nullptr, erow, s, false, &nbp, part)))
      return fail(rc);
    if (!part) part = m->partial;
    hipEvent_t ev;
    prof_begin(m, PROF_STEP, s, &ev);
    double *kin = part + nbp * PARTIAL_COLS;  // after the pair partials
    int64_t nkin = 0;
    // the previous step's velocity rescaling (side stream) precedes this leapfrog
    rc = (overlap && nvt && st >= 1) ? check_hip(hipStreamWaitEvent(s, m->ev_red[(st - 1) & 1], 0), "hipStreamWaitEvent")
                                     : MD_OK;
    if (!rc)
      rc = launch_leapfrog(m, pos, vel, quat, angmom, m->host.ncomp > 1 ? comp : nullptr, N, box, dt, m->force,
                           m->torque, kin, &nkin, s);
    // energies row: U, W from the pair partials and K_trans, K_rot from the leapfrog's, in one
    // reduction (skipped when neither energies nor the thermostat need it); the thermostat then
    // rescales the new half-step velocities from the reduced K(t) and degrees of freedom
    if (!rc && overlap) {
      rc = check_hip(hipEventRecord(m->ev_leap[slot], s), "hipEventRecord");
      if (!rc) rc = check_hip(hipStreamWaitEvent(m->side, m->ev_leap[slot], 0), "hipStreamWaitEvent");
      if (!rc) rc = launch_reduce_forces(m, nbp, part, m->uw + 8, nullptr, erow, m->side, kin, nkin);
      if (!rc && nvt)
        rc = launch_rescale(m, vel, angmom, m->host.ncomp > 1 ? comp : nullptr, N, m->uw + 13, m->T_target, m->side);
      if (!rc) rc = check_hip(hipEventRecord(m->ev_red[slot], m->side), "hipEventRecord");
      if (!rc) last_red = slot;
    } else if (!rc && (erow || nvt)) {
      rc = launch_reduce_forces(m, nbp, part, m->uw + 8, nullptr, erow, s, kin, nkin);
      if (!rc && nvt)
        rc = launch_rescale(m, vel, angmom, m->host.ncomp > 1 ? comp : nullptr, N, m->uw + 13, m->T_target, s);
    }
    prof_end(m, PROF_STEP, s, ev);
    if (rc) {
      // a reduction queued on the side stream whose event was not recorded: wait for all of it
      if (overlap && m->side) (void)hipStreamSynchronize(m->side);
      return fail(rc);
    }
  }
  // the caller's stream sees every reduction of this call
  if (overlap && (rc = check_hip(hipStreamWaitEvent(s, m->ev_red[(nsteps - 1) & 1], 0), "hipStreamWaitEvent")))
    return rc;
  return sync_check(m, s);
}

int md_set_thermostat(md_model *m, double T_target) {
  if (!m) return set_error(MD_EINVAL, "md_set_thermostat: NULL model");
  if (!std::isfinite(T_target)) return set_error(MD_ENONFINITE, "md_set_thermostat: T_target not finite");
  if (T_target < 0.0) return set_error(MD_EINVAL, "md_set_thermostat: T_target < 0");
  m->T_target = T_target;
  return MD_OK;
}

int md_long_range_correction(const md_component_desc *comps, int32_t ncomp, const double *xi, const double *eta,
                             double rc, uint32_t flags, const int64_t *counts, const double box[3], double *u_lrc,
                             double *w_lrc) {
  if (!comps || !counts || !box || !u_lrc || !w_lrc)
    return set_error(MD_EINVAL, "md_long_range_correction: NULL argument");
  if (ncomp < 1) return set_error(MD_EINVAL, "md_long_range_correction: ncomp < 1");
  if (ncomp > MD_MAX_COMP) return set_error(MD_ECOMP, "md_long_range_correction: ncomp exceeds MD_MAX_COMP");
  if (!std::isfinite(rc)) return set_error(MD_ENONFINITE, "md_long_range_correction: r_c not finite");
  if (!(rc > 0.0)) return set_error(MD_EINVAL, "md_long_range_correction: r_c <= 0");
  if (flags & ~(MD_LJ_SHIFT | MD_CHECK | MD_HALF_SHELL | MD_SUBCELLS))
    return set_error(MD_EINVAL, "md_long_range_correction: unknown flag");
  double V = 1.0;
  for (int k = 0; k < 3; ++k) {
    if (!std::isfinite(box[k])) return set_error(MD_ENONFINITE, "md_long_range_correction: box not finite");
    if (!(box[k] > 0.0)) return set_error(MD_EINVAL, "md_long_range_correction: box <= 0");
    V *= box[k];
  }
  for (int c = 0; c < ncomp; ++c) {
    const md_component_desc &d = comps[c];
    if (counts[c] < 0) return set_error(MD_EINVAL, "md_long_range_correction: negative count");
    if (d.n_lj < 0) return set_error(MD_EINVAL, "md_long_range_correction: negative site count");
    if (d.n_lj > MD_MAX_LJ) return set_error(MD_ECOMP, "md_long_range_correction: site count exceeds the compiled limits");
    if (d.n_lj && (!d.lj_eps || !d.lj_sigma)) return set_error(MD_EINVAL, "md_long_range_correction: NULL site table");
    for (int a = 0; a < d.n_lj; ++a) {
      if (!std::isfinite(d.lj_eps[a]) || !std::isfinite(d.lj_sigma[a]))
        return set_error(MD_ENONFINITE, "md_long_range_correction: non-finite site table entry");
      if (!(d.lj_eps[a] > 0.0) || !(d.lj_sigma[a] > 0.0))
        return set_error(MD_EINVAL, "md_long_range_correction: LJ epsilon and sigma must be > 0");
    }
  }
  for (int a = 0; a < ncomp * ncomp; ++a) {
    const double x = xi ? xi[a] : 1.0, e = eta ? eta[a] : 1.0;
    if (!std::isfinite(x) || !std::isfinite(e)) return set_error(MD_ENONFINITE, "md_long_range_correction: xi/eta not finite");
    if (!(x > 0.0) || !(e > 0.0)) return set_error(MD_EINVAL, "md_long_range_correction: xi/eta must be > 0");
  }
  double U = 0.0, W = 0.0;
  if (!(flags & MD_LJ_SHIFT)) {
    const double pi = 3.14159265358979323846;
    for (int A = 0; A < ncomp; ++A)
      for (int B = 0; B < ncomp; ++B) {
        const double dens = 2.0 * pi * (double)counts[A] * (double)counts[B] / V;
        const double x = xi ? xi[A * ncomp + B] : 1.0, e = eta ? eta[A * ncomp + B] : 1.0;
        for (int a = 0; a < comps[A].n_lj; ++a)
          for (int b = 0; b < comps[B].n_lj; ++b) {
            const double eps = x * std::sqrt(comps[A].lj_eps[a] * comps[B].lj_eps[b]);
            const double sig = e * 0.5 * (comps[A].lj_sigma[a] + comps[B].lj_sigma[b]);
            const double s3 = sig * sig * sig / (rc * rc * rc);
            const double e4s3 = 4.0 * eps * sig * sig * sig;
            U += dens * e4s3 * (s3 * s3 * s3 / 9.0 - s3 / 3.0);
            W += dens * e4s3 * (4.0 * s3 * s3 * s3 / 3.0 - 2.0 * s3);
          }
      }
  }
  *u_lrc = U;
  *w_lrc = W;
  return MD_OK;
}

int md_forces_adjoint(md_model *m, const md_cells *c, int precision, double gU, double *dpos, double *dquat,
                      double *dparams, void *stream) {
  if (!m || !c || !dpos) return set_error(MD_EINVAL, "md_forces_adjoint: NULL argument");
  if (precision != MD_FP64 && precision != MD_FP32) return set_error(MD_EINVAL, "md_forces_adjoint: bad precision");
  if (!std::isfinite(gU)) return set_error(MD_ENONFINITE, "md_forces_adjoint: gU not finite");
  if (!c->built || c->model != m) return set_error(MD_EINVAL, "md_forces_adjoint: cells not built with this model");
  hipStream_t s = (hipStream_t)stream;
  m->last_stream = s;
  int rc;
  if (m->single_site) {
    // One LJ site at the centre: gU dU/dr_i = -gU F_i, and the parameter gradients follow from one
    // force evaluation (U is linear in eps; sigma dU/dsigma is the virial minus the shift's share;
    // the offset gradient sum_i dU/dr_i vanishes), so the force kernel serves as the adjoint.
    double *uw5 = m->uw + 24;
    int64_t *np = (int64_t *)(m->uw + 32);
    hipEvent_t ev;
    prof_begin(m, PROF_ADJ, s, &ev);
    rc = forces_impl(m, c, precision, dpos, nullptr, nullptr, nullptr, nullptr, uw5, np, nullptr, s, dparams != nullptr);
    if (!rc) rc = launch_lj_adjoint_finish(m, dpos, c->N, gU, uw5, np, dparams, s);
    if (!rc && dquat) rc = launch_fill_f64(dquat, 4 * c->N, 0.0, s);
    prof_end(m, PROF_ADJ, s, ev);
    if (rc) return rc;
    return sync_check(m, s);
  }
  const int64_t nb = pair_blocks(c->ncell);
  double *pg = nullptr;
  if (dparams && m->nparam > 0) {
    if ((rc = grow(m->pgrad, m->cap_pgrad, nb * m->nparam, "param partials"))) return rc;
    pg = m->pgrad;
  }
  AdjOut o{gU, dpos, dquat, pg};
  int64_t nblocks = 0;
  hipEvent_t ev;
  prof_begin(m, PROF_ADJ, s, &ev);
  rc = launch_adjoint(m, c, precision, o, m->single_site ? nullptr : c->squat, s, &nblocks);
  if (!rc && pg) rc = launch_reduce(m, nblocks, (int)m->nparam, pg, dparams, s);
  prof_end(m, PROF_ADJ, s, ev);
  if (rc) return rc;
  return sync_check(m, s);
}

int md_status(md_model *m, int32_t *flags) {
  if (!m || !flags) return set_error(MD_EINVAL, "md_status: NULL argument");
  int rc = check_hip(hipStreamSynchronize(m->last_stream), "hipStreamSynchronize");
  if (rc) return rc;
  rc = check_hip(hipMemcpy(flags, m->status, sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy(status)");
  if (rc) return rc;
  if ((rc = launch_fill_i32(m->status, 1, 0, m->last_stream))) return rc;
  return check_hip(hipStreamSynchronize(m->last_stream), "hipStreamSynchronize");
}

int md_profile(md_model *m, int enable) {
  if (!m) return set_error(MD_EINVAL, "md_profile: NULL model");
  for (auto &e : m->events) (void)hipEventDestroy(e.a), (void)hipEventDestroy(e.b);
  m->events.clear();
  for (int k = 0; k < 4; ++k) m->prof_ms[k] = 0.0, m->prof_n[k] = 0;
  m->profiling = enable != 0;
  return MD_OK;
}

int md_profile_read(md_model *m, const char *group, double *total_ms, int64_t *launches) {
  if (!m || !group || !total_ms || !launches) return set_error(MD_EINVAL, "md_profile_read: NULL argument");
  int g = -1;
  if (!std::strcmp(group, "pair")) g = PROF_PAIR;
  else if (!std::strcmp(group, "build")) g = PROF_BUILD;
  else if (!std::strcmp(group, "step")) g = PROF_STEP;
  else if (!std::strcmp(group, "adjoint")) g = PROF_ADJ;
  if (g < 0) return set_error(MD_EINVAL, "md_profile_read: unknown group");
  for (auto &e : m->events) {
    int rc = check_hip(hipEventSynchronize(e.b), "hipEventSynchronize");
    if (rc) return rc;
    float ms = 0.0f;
    rc = check_hip(hipEventElapsedTime(&ms, e.a, e.b), "hipEventElapsedTime");
    if (rc) return rc;
    m->prof_ms[e.group] += ms;
    m->prof_n[e.group] += 1;
    (void)hipEventDestroy(e.a), (void)hipEventDestroy(e.b);
  }
  m->events.clear();
  *total_ms = m->prof_ms[g];
  *launches = m->prof_n[g];
  return MD_OK;
}

}  // extern "C"
