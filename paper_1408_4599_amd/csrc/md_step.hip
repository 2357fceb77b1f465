// Leapfrog integration (Sec. 3, Eqs. 2-5): translational kick-drift with periodic wrap and,
// for molecules with inertia, Fincham's rotational leapfrog on quaternions with the space-frame
// angular momentum.  HBM-bound (~120 B/molecule translational, one thread per Cartesian component;
// ~+136 B rotational), with per-block kinetic-energy partials reduced deterministically.

#include "md_internal.h"

namespace mdcell {
namespace {

struct LeapArgs {
  double *pos, *vel, *quat, *angmom;
  const int32_t *comp;
  int64_t N;
  double Lx, Ly, Lz, dt;
  const double *force, *torque;
  const ModelDev *md;
  double *partial;  // [rows][KIN_COLS]: K_trans, K_rot, rotational dof block partials
};

__device__ __forceinline__ void rotmat(const double *q, double A[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  A[0][0] = w * w + x * x - y * y - z * z, A[0][1] = 2.0 * (x * y - w * z), A[0][2] = 2.0 * (x * z + w * y);
  A[1][0] = 2.0 * (x * y + w * z), A[1][1] = w * w - x * x + y * y - z * z, A[1][2] = 2.0 * (y * z - w * x);
  A[2][0] = 2.0 * (x * z - w * y), A[2][1] = 2.0 * (y * z + w * x), A[2][2] = w * w - x * x - y * y + z * z;
}

// Body-frame angular velocity w_b = I^-1 A(q)^T j (I_k^-1 = 0 on an axis with I_k = 0).
__device__ __forceinline__ void omega_body(const double *q, const double *j, const double *inv_I, double *wb) {
  double A[3][3];
  rotmat(q, A);
#pragma unroll
  for (int k = 0; k < 3; ++k) wb[k] = (A[0][k] * j[0] + A[1][k] * j[1] + A[2][k] * j[2]) * inv_I[k];
}

// out = q + h * (1/2) qr (x) (0, w_b)
__device__ __forceinline__ void q_advance(const double *q, const double *qr, const double *w, double h, double *out) {
  const double d0 = -qr[1] * w[0] - qr[2] * w[1] - qr[3] * w[2];
  const double d1 = qr[0] * w[0] + qr[2] * w[2] - qr[3] * w[1];
  const double d2 = qr[0] * w[1] - qr[1] * w[2] + qr[3] * w[0];
  const double d3 = qr[0] * w[2] + qr[1] * w[1] - qr[2] * w[0];
  out[0] = q[0] + h * 0.5 * d0, out[1] = q[1] + h * 0.5 * d1, out[2] = q[2] + h * 0.5 * d2, out[3] = q[3] + h * 0.5 * d3;
}

__device__ __forceinline__ void q_normalise(double *q) {
  const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  q[0] /= n, q[1] /= n, q[2] /= n, q[3] /= n;
}

// Fixed-order block sums (wave shuffles, then the four wave sums in order) of the values of
// columns col .. col + n - 1 into partial[row][...]; the other columns of the row are set to zero.
template <int n>
__device__ __forceinline__ void block_partial(const double (&v)[n], double *partial, int64_t row, int col) {
  __shared__ double sk[n][4];
  double x[n];
#pragma unroll
  for (int c = 0; c < n; ++c) {
    x[c] = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x[c] += __shfl_xor(x[c], o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < n; ++c) sk[c][w] = x[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    double *r = partial + KIN_COLS * row;
    for (int c = 0; c < KIN_COLS; ++c) r[c] = 0.0;
    for (int c = 0; c < n; ++c) r[col + c] = ((sk[c][0] + sk[c][1]) + sk[c][2]) + sk[c][3];
  }
}

// Translational kick-drift over the 3N Cartesian components, LF_PER per thread (block b takes
// components [b 256 LF_PER, (b + 1) 256 LF_PER), thread j components j, j + 256, ...: every
// access coalesced, LF_PER loads in flight per thread): v += dt F / m, r = wrap(r + dt v); K_trans
// from the mid-step velocity.
constexpr int LF_PER = 4;
__global__ __launch_bounds__(256) void k_leapfrog_trans(LeapArgs a) {
  const int64_t base = (int64_t)blockIdx.x * (256 * LF_PER) + threadIdx.x;
  double kt = 0.0;
#pragma unroll
  for (int r = 0; r < LF_PER; ++r) {
    const int64_t t = base + 256 * r;
    if (t < 3 * a.N) {
      const int64_t i = t / 3;
      const int k = (int)(t - 3 * i);
      int c = a.comp ? a.comp[i] : 0;
      if (c < 0 || c >= a.md->ncomp) c = 0;
      const double mass = a.md->comp[c].mass;
      const double vold = a.vel[t];
      const double vnew = vold + a.dt * a.force[t] / mass;
      const double vmid = 0.5 * (vold + vnew);
      kt += 0.5 * mass * (vmid * vmid);
      a.vel[t] = vnew;
      a.pos[t] = wrap1(a.pos[t] + a.dt * vnew, k == 0 ? a.Lx : (k == 1 ? a.Ly : a.Lz));
    }
  }
  const double kv[1] = {kt};
  block_partial(kv, a.partial, blockIdx.x, 0);
}

// Rotational leapfrog (Fincham), one thread per molecule; K_rot at the half step.  Block partials
// go to rows row0 + blockIdx.x.
__global__ __launch_bounds__(256) void k_leapfrog_rot(LeapArgs a, int64_t row0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double kr = 0.0, fr = 0.0;
  if (i < a.N) {
    int c = a.comp ? a.comp[i] : 0;
    if (c < 0 || c >= a.md->ncomp) c = 0;
    const CompDev &cd = a.md->comp[c];
    if (cd.rotates) {
      fr = (double)((cd.inertia[0] > 0.0) + (cd.inertia[1] > 0.0) + (cd.inertia[2] > 0.0));
      double q[4], jm[3], tq[3];
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = a.quat[4 * i + k];
#pragma unroll
      for (int k = 0; k < 3; ++k) jm[k] = a.angmom[3 * i + k], tq[k] = a.torque[3 * i + k];
      double jt[3], wb[3], qh[4], jn[3], wbh[3], qn[4];
#pragma unroll
      for (int k = 0; k < 3; ++k) jt[k] = jm[k] + 0.5 * a.dt * tq[k];
      omega_body(q, jt, cd.inv_inertia, wb);
#pragma unroll
      for (int k = 0; k < 3; ++k) kr += 0.5 * wb[k] * wb[k] * cd.inertia[k];
      q_advance(q, q, wb, 0.5 * a.dt, qh);
      q_normalise(qh);
#pragma unroll
      for (int k = 0; k < 3; ++k) jn[k] = jm[k] + a.dt * tq[k];
      omega_body(qh, jn, cd.inv_inertia, wbh);
      q_advance(q, qh, wbh, a.dt, qn);
      q_normalise(qn);
#pragma unroll
      for (int k = 0; k < 4; ++k) a.quat[4 * i + k] = qn[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) a.angmom[3 * i + k] = jn[k];
    }
  }
  const double kv[2] = {kr, fr};
  block_partial(kv, a.partial, row0 + blockIdx.x, 1);
}

// Velocity rescaling (NVT): v *= beta for every component, j *= beta for molecules with inertia,
// beta = sqrt(f T_target / (2 K)), f = 3 N + kin[2], K = kin[0] + kin[1] (beta = 1 if K = 0).
// One thread per Cartesian component.
__global__ __launch_bounds__(256) void k_rescale(double *vel, double *angmom, const int32_t *comp,
                                                 const ModelDev *md, int64_t N, const double *kin,
                                                 double T_target) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * N) return;
  const double K = kin[0] + kin[1];
  const double f = 3.0 * (double)N + kin[2];
  const double beta = K > 0.0 ? sqrt(0.5 * f * T_target / K) : 1.0;
  vel[t] *= beta;
  if (angmom) {
    int c = comp ? comp[t / 3] : 0;
    if (c < 0 || c >= md->ncomp) c = 0;
    if (md->comp[c].rotates) angmom[t] *= beta;
  }
}

}  // namespace

int launch_leapfrog(md_model *m, double *pos, double *vel, double *quat, double *angmom, const int32_t *comp,
                    int64_t N, const double box[3], double dt, const double *force, const double *torque,
                    double *kin_rows, int64_t *kin_nrows, hipStream_t s) {
  const int64_t nt = (3 * N + 256 * LF_PER - 1) / (256 * LF_PER);
  const bool rot = !m->single_site && quat && angmom;
  const int64_t nr = rot ? (N + 255) / 256 : 0;
  LeapArgs a{pos, vel, rot ? quat : nullptr, rot ? angmom : nullptr, comp, N, box[0], box[1],
             box[2], dt, force, torque, m->dev, kin_rows};
  k_leapfrog_trans<<<(unsigned)nt, 256, 0, s>>>(a);
  if (rot) k_leapfrog_rot<<<(unsigned)nr, 256, 0, s>>>(a, nt);
  *kin_nrows = nt + nr;
  return check_hip(hipGetLastError(), "k_leapfrog");
}

int launch_rescale(md_model *m, double *vel, double *angmom, const int32_t *comp, int64_t N, const double *kin,
                   double T_target, hipStream_t s) {
  const bool rot = !m->single_site && angmom;
  k_rescale<<<(unsigned)((3 * N + 255) / 256), 256, 0, s>>>(vel, rot ? angmom : nullptr, comp, m->dev, N, kin,
                                                            T_target);
  return check_hip(hipGetLastError(), "k_rescale");
}

}  // namespace mdcell
