// Adjoint of the total potential energy U (Sec. 2 interaction models over the linked-cell pair
// set of Sec. 3): gU dU/d(COM positions), gU dU/d(raw quaternion components) and
// gU dU/d(epsilon, sigma, site offsets, charges, dipole and quadrupole moments).
//
// Recomputation backward: the cell traversal of the force kernel is run again and no pair list is
// stored.  Each molecule lane accumulates, over all its partners, dU/d(world position) of each of
// its sites, dU/d(world axis) of each dipole / quadrupole and the derivative of the pair energies
// with respect to its own sites' parameters (each pair end credits only its own sites, so every
// parameter dependence of every pair is counted once).  Then per molecule:
//   dU/dr_i = sum_a dU/dx_ia;
//   dU/dq_i = sum over site vectors v (body offsets d_a, body axes e_a) of J_v(q)^T g_v with
//             A(q) v = (w^2 - |u|^2) v + 2 (u.v) u + 2 w (u x v), q = (w, u);
//   dU/dd_a = A(q_i)^T dU/dx_ia, summed over the molecules of the component.
// Parameter partials are reduced per block in a fixed order, then over blocks by the
// deterministic column reduction.

#include "md_device.h"

namespace mdcell {
namespace {

// PRM: the parameter partials (peps, psig, pmom) are accumulated; without dU/d(parameters) they
// are left out of the pair loop.
template <int SL, int SC, int SD, int SQ, bool PRM = true> struct AdjAcc {
  static constexpr int NSITE = SL + SC + SD + SQ;
  static constexpr int NAX = SD + SQ > 0 ? SD + SQ : 1;
  static constexpr int NMOM = SC + SD + SQ > 0 ? SC + SD + SQ : 1;
  double gs[NSITE][3];  // dU/d(site position), world frame: LJ, charges, dipoles, quadrupoles
  double ga[NAX][3];    // dU/d(site axis), world frame: dipoles, quadrupoles
  double peps[SL], psig[SL];
  double pmom[NMOM];    // dU/d(moment): charges, dipoles, quadrupoles
  int n;
};

template <int KA, int KB, int SL, int SC, int SD, int SQ, bool MIX, typename R, bool PRM>
__device__ __forceinline__ void adj_elec_group(const CompDev &A, const CompDev &B, const R (*vi)[3], const R *vj,
                                               R dx, R dy, R dz, R krc3, AdjAcc<SL, SC, SD, SQ, PRM> &acc) {
#pragma clang fp contract(fast)  // products and sums fused where the compiler can (pair algebra only)
  using S = Slots<SL, SC, SD, SQ>;
  constexpr int NA = KA == KIND_CHG ? SC : (KA == KIND_DIP ? SD : SQ);
  constexpr int NB = KB == KIND_CHG ? SC : (KB == KIND_DIP ? SD : SQ);
  constexpr int OA = KA == KIND_CHG ? S::chg : (KA == KIND_DIP ? S::dip : S::quad);
  constexpr int OB = KB == KIND_CHG ? S::chg : (KB == KIND_DIP ? S::dip : S::quad);
  constexpr int EA = KA == KIND_DIP ? S::dipax : (KA == KIND_QUAD ? S::quadax : 0);
  constexpr int EB = KB == KIND_DIP ? S::dipax : (KB == KIND_QUAD ? S::quadax : 0);
  constexpr int SA = KA == KIND_CHG ? SL : (KA == KIND_DIP ? SL + SC : SL + SC + SD);  // site index base
  constexpr int XA = KA == KIND_DIP ? 0 : SD;                                          // axis index base
  constexpr int MA = KA == KIND_CHG ? 0 : (KA == KIND_DIP ? SC : SC + SD);             // moment index base
  const int na = MIX ? (KA == KIND_CHG ? A.n_chg : (KA == KIND_DIP ? A.n_dip : A.n_quad)) : NA;
  const int nb = MIX ? (KB == KIND_CHG ? B.n_chg : (KB == KIND_DIP ? B.n_dip : B.n_quad)) : NB;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    if (a >= na) break;
    const R ma = (R)(KA == KIND_CHG ? A.chg_q[a] : (KA == KIND_DIP ? A.dip_mu[a] : A.quad_Q[a]));
    const R *oa = vi[OA + a];
    const R *ea = vi[EA + a];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b >= nb) break;
      const R mb = (R)(KB == KIND_CHG ? B.chg_q[b] : (KB == KIND_DIP ? B.dip_mu[b] : B.quad_Q[b]));
      const R *ob = vj + 3 * (OB + b);
      const R *eb = vj + 3 * (EB + b);
      const R rx = dx + oa[0] - ob[0], ry = dy + oa[1] - ob[1], rz = dz + oa[2] - ob[2];
      const R r2 = fma(rz, rz, fma(ry, ry, rx * rx));
      const R ir = rsq_nr<R>(r2);
      const R rh[3] = {rx * ir, ry * ir, rz * ir};
      const R ci = (KA != KIND_CHG) ? fma(ea[2], rh[2], fma(ea[1], rh[1], ea[0] * rh[0])) : (R)0;
      const R cj = (KB != KIND_CHG) ? fma(eb[2], rh[2], fma(eb[1], rh[1], eb[0] * rh[0])) : (R)0;
      const R cij = (KA != KIND_CHG && KB != KIND_CHG) ? fma(ea[2], eb[2], fma(ea[1], eb[1], ea[0] * eb[0])) : (R)0;
      const Unit<R> t = unit_terms<KA, KB, R>(ir, ci, cj, cij, krc3);
      const R pm = ma * mb;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        R g = t.tr * rh[k];
        if constexpr (KA != KIND_CHG) g += t.ti * (ea[k] - ci * rh[k]) * ir;
        if constexpr (KB != KIND_CHG) g += t.tj * (eb[k] - cj * rh[k]) * ir;
        acc.gs[SA + a][k] += (double)(pm * g);
        if constexpr (KA != KIND_CHG) {
          R ge = t.ti * rh[k];
          if constexpr (KB != KIND_CHG) ge += t.tij * eb[k];
          acc.ga[XA + a][k] += (double)(pm * ge);
        }
      }
      if constexpr (PRM) acc.pmom[MA + a] += (double)(mb * t.t);
    }
  }
}

template <int SL, int SC, int SD, int SQ, bool MIX, typename R, bool PRM>
__device__ __forceinline__ void adj_pair(const ModelDev *__restrict__ md, int ci, int cj, const R (*vi)[3],
                                         const R *vj, R dx, R dy, R dz, AdjAcc<SL, SC, SD, SQ, PRM> &acc) {
#pragma clang fp contract(fast)
  const CompDev &A = md->comp[ci];
  const CompDev &B = md->comp[cj];
  const int nla = MIX ? A.n_lj : SL, nlb = MIX ? B.n_lj : SL;
#pragma unroll
  for (int a = 0; a < SL; ++a) {
    if (a >= nla) break;
#pragma unroll
    for (int b = 0; b < SL; ++b) {
      if (b >= nlb) break;
      const LJPair &p = md->lj[ci][cj][a][b];
      const R *ob = vj + 3 * b;
      const R rx = dx + vi[a][0] - ob[0], ry = dy + vi[a][1] - ob[1], rz = dz + vi[a][2] - ob[2];
      const R r2 = fma(rz, rz, fma(ry, ry, rx * rx));
      const R ir2 = rcp_nr<R>(r2);
      const R s2 = (R)p.sig2 * ir2;
      const R s6 = s2 * s2 * s2;
      const R s12 = s6 * s6;
      // dU/dR = -24 eps (2 s^12 - s^6) / r^2 R
      const R gsc = -((R)p.eps24 * ir2) * (s6 * fma((R)2, s6, (R)-1));
      acc.gs[a][0] += (double)(gsc * rx), acc.gs[a][1] += (double)(gsc * ry), acc.gs[a][2] += (double)(gsc * rz);
      if constexpr (PRM) {
        const double u = (double)((R)p.eps4 * (s12 - s6)) - p.shift;
        acc.peps[a] += u * p.pe;
        acc.psig[a] += p.ps * ((double)((R)12 * s12 - (R)6 * s6) - p.csh);
      }
    }
  }
  if constexpr (SC + SD + SQ > 0) {
    const R krc3 = (R)md->kappa_rc3;
    if constexpr (SC > 0) {
      adj_elec_group<KIND_CHG, KIND_CHG, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
      if constexpr (SD > 0) {
        adj_elec_group<KIND_CHG, KIND_DIP, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
        adj_elec_group<KIND_DIP, KIND_CHG, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
      }
      if constexpr (SQ > 0) {
        adj_elec_group<KIND_CHG, KIND_QUAD, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
        adj_elec_group<KIND_QUAD, KIND_CHG, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
      }
    }
    if constexpr (SD > 0) {
      adj_elec_group<KIND_DIP, KIND_DIP, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
      if constexpr (SQ > 0) {
        adj_elec_group<KIND_DIP, KIND_QUAD, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
        adj_elec_group<KIND_QUAD, KIND_DIP, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
      }
    }
    if constexpr (SQ > 0) adj_elec_group<KIND_QUAD, KIND_QUAD, SL, SC, SD, SQ, MIX>(A, B, vi, vj, dx, dy, dz, krc3, acc);
  }
}

// J_v(q)^T g for A(q) v = (w^2 - |u|^2) v + 2 (u.v) u + 2 w (u x v), added into dq.
__device__ __forceinline__ void quat_vjp(const double *q, const double *v, const double *g, double *dq) {
  const double w = q[0], ux = q[1], uy = q[2], uz = q[3];
  const double gv = g[0] * v[0] + g[1] * v[1] + g[2] * v[2];
  const double gu = g[0] * ux + g[1] * uy + g[2] * uz;
  const double uv = ux * v[0] + uy * v[1] + uz * v[2];
  const double uxv[3] = {uy * v[2] - uz * v[1], uz * v[0] - ux * v[2], ux * v[1] - uy * v[0]};
  const double vxg[3] = {v[1] * g[2] - v[2] * g[1], v[2] * g[0] - v[0] * g[2], v[0] * g[1] - v[1] * g[0]};
  dq[0] += 2.0 * w * gv + 2.0 * (g[0] * uxv[0] + g[1] * uxv[1] + g[2] * uxv[2]);
  const double u[3] = {ux, uy, uz};
#pragma unroll
  for (int k = 0; k < 3; ++k) dq[1 + k] += -2.0 * gv * u[k] + 2.0 * gu * v[k] + 2.0 * uv * g[k] + 2.0 * w * vxg[k];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int SL, int SC, int SD, int SQ, bool PRM>
__device__ __forceinline__ void acc_zero(AdjAcc<SL, SC, SD, SQ, PRM> &acc) {
  using Acc = AdjAcc<SL, SC, SD, SQ, PRM>;
#pragma unroll
  for (int a = 0; a < Acc::NSITE; ++a) acc.gs[a][0] = acc.gs[a][1] = acc.gs[a][2] = 0.0;
#pragma unroll
  for (int a = 0; a < Acc::NAX; ++a) acc.ga[a][0] = acc.ga[a][1] = acc.ga[a][2] = 0.0;
#pragma unroll
  for (int a = 0; a < SL; ++a) acc.peps[a] = acc.psig[a] = 0.0;
#pragma unroll
  for (int a = 0; a < Acc::NMOM; ++a) acc.pmom[a] = 0.0;
  acc.n = 0;
}

// Add the slices of molecule lane l (lanes l + s hc, s = 1 .. NS - 1) to lane l, in slice order.
template <int SL, int SC, int SD, int SQ, bool PRM>
__device__ __forceinline__ void acc_gather(AdjAcc<SL, SC, SD, SQ, PRM> &acc, int hc, int NS) {
  using Acc = AdjAcc<SL, SC, SD, SQ, PRM>;
  const int lane = threadIdx.x & 63;
  const bool dst = lane < hc;
  auto add = [&](double &v, int src) {
    const double w = __shfl(v, src);
    if (dst) v += w;
  };
  for (int s2 = 1; s2 < NS; ++s2) {
    const int src = lane + s2 * hc;  // meaningful for lane < hc
#pragma unroll
    for (int a = 0; a < Acc::NSITE; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) add(acc.gs[a][k], src);
#pragma unroll
    for (int a = 0; a < Acc::NAX; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) add(acc.ga[a][k], src);
#pragma unroll
    for (int a = 0; a < SL && PRM; ++a) add(acc.peps[a], src), add(acc.psig[a], src);
#pragma unroll
    for (int a = 0; a < Acc::NMOM && PRM; ++a) add(acc.pmom[a], src);
    const int n = __shfl(acc.n, src);
    if (dst) acc.n += n;
  }
}

// Parameter-gradient slots of one molecule in a compile-time layout (per LJ site: eps, sigma,
// offset xyz; per charge / dipole / quadrupole: moment, offset xyz) and their ABI columns.
template <int SL, int SC, int SD, int SQ> struct PSlots {
  static constexpr int np = 5 * SL + 4 * (SC + SD + SQ);
  static constexpr int chg = 5 * SL, dip = 5 * SL + 4 * SC, quad = 5 * SL + 4 * (SC + SD);
};

// One block of W wavefronts per home cell, staged through shared LDS windows of CAP molecules as
// in the force kernel; pass 1 lists the COM-cutoff hits, pass 2 recomputes each listed pair's
// site terms into the lane's adjoint accumulators (the hits of a molecule split evenly over its
// slice lanes), slices are then added in a fixed order.
// PRM: parameter gradients wanted (o.pgrad given); without them the pair loop leaves out the
// parameter partials.
template <typename R, int SL, int SC, int SD, int SQ, bool MIX, int CAP, int W, bool PRM>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(MIX ? 1 : 3))) void k_adjoint(
    CellsDev c, const ModelDev *__restrict__ md, const double *quat, double rc2, AdjOut o) {
  using S = Slots<SL, SC, SD, SQ>;
  using Acc = AdjAcc<SL, SC, SD, SQ, PRM>;
  using PS = PSlots<SL, SC, SD, SQ>;
  constexpr int NV = S::nv;
  constexpr int LCAP = 32;
  constexpr int NB = !PRM ? 1 : (MIX ? 256 : PS::np);
  static_assert(CAP <= 256, "list entries are bytes");
  __shared__ double jp[CAP * 3 + 48];  // slack: the walk reads up to 2 NS - 1 slots past the window
  __shared__ R jv[CAP][NV * 3];
  __shared__ int jc_[MIX ? CAP : 1];
  __shared__ unsigned char lists[W][LCAP * 64];
  __shared__ int scnts[W][64];
  __shared__ NbTable nb;
  __shared__ double bsums[W][NB];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  unsigned char *list = lists[wave];
  int *scnt = scnts[wave];
  double *bsum = bsums[wave];
  const int cell = xcd_remap(blockIdx.x, gridDim.x);
  const int hs = cell < c.ncell ? c.cell_start[cell] : 0;
  const int hn = cell < c.ncell ? __builtin_amdgcn_readfirstlane(c.cell_start[cell + 1] - hs) : 0;
  const int ncol = md->nparam;
  if (o.pgrad)
    for (int k = lane; k < ncol; k += 64) bsum[k] = 0.0;
  if (hn > 0) {
    if (tid < 64) build_nb(c, cell, nb);
    __syncthreads();
    const int M = nb.off[27];
    const int self0 = nb.off[13];
    for (int ic = 0; ic < hn; ic += 64 * W) {
      // this round's molecules, split evenly over the wavefronts (wave-uniform)
      const int rem = min(64 * W, hn - ic), base = rem / W, extra = rem % W;
      const int hc = base + (wave < extra ? 1 : 0);
      const int i0 = ic + wave * base + min(wave, extra);
      const int NS = hc > 0 ? min(8, 64 / hc) : 1;
      const int il = hc > 0 ? lane % hc : 0, sl = hc > 0 ? lane / hc : NS;
      const bool act = sl < NS;
      const int sla = act ? sl : 0;
      const int iloc = i0 + il;
      double xi = 1e30, yi = 1e30, zi = 1e30;  // idle lanes: no candidate is within the cutoff
      R vi[NV][3];
      int ci = 0;
#pragma unroll
      for (int k = 0; k < NV; ++k) vi[k][0] = vi[k][1] = vi[k][2] = (R)0;
      {
        const int sidx = hs + (hc > 0 ? iloc : 0);
        if (act) xi = c.sx[sidx], yi = c.sy[sidx], zi = c.sz[sidx];
        if (MIX) ci = c.scomp[sidx];
        {
          const double *v = c.svec + (int64_t)sidx * NV * 3;
#pragma unroll
          for (int k = 0; k < NV; ++k) vi[k][0] = (R)v[3 * k], vi[k][1] = (R)v[3 * k + 1], vi[k][2] = (R)v[3 * k + 2];
        }
      }
      Acc acc;
      acc_zero(acc);
      int cnt = 0;
      unsigned char *mylist = list + lane;
      auto flush = [&]() {
        scnt[lane] = cnt;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (act) {
          int H = 0;
          for (int s2 = 0; s2 < NS; ++s2) H += scnt[il + s2 * hc];
          const int q0 = H * sl / NS, q1 = H * (sl + 1) / NS;
          int sp = 0, j = q0, csp = scnt[il];
          for (int q = q0; q < q1; ++q, ++j) {
            while (j >= csp) j -= csp, ++sp, csp = scnt[il + sp * hc];
            const int u = list[il + sp * hc + 64 * j];
            const double dx = xi - jp[3 * u], dy = yi - jp[3 * u + 1], dz = zi - jp[3 * u + 2];
            const int cj = MIX ? jc_[u] : 0;
            adj_pair<SL, SC, SD, SQ, MIX, R>(md, ci, cj, vi, jv[u], (R)dx, (R)dy, (R)dz, acc);
            acc.n += 1;
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
          if (MIX) jc_[t] = c.scomp[src];
          {
            const double *v = c.svec + (int64_t)src * NV * 3;
#pragma unroll
            for (int q = 0; q < NV * 3; ++q) jv[t][q] = (R)v[q];
          }
        }
        __syncthreads();
        if (hc > 0) {
          const int self = self0 + iloc - jc;  // window slot of the molecule itself (may be outside)
          int kb = 0;
          while (true) {
            for (; kb < mj && !__any(cnt > LCAP - 2); kb += 2 * NS) {
              const int ta = kb + sla, tb = ta + NS;
              const double ax = xi - jp[3 * ta], ay = yi - jp[3 * ta + 1], az = zi - jp[3 * ta + 2];
              const double bx_ = xi - jp[3 * tb], by_ = yi - jp[3 * tb + 1], bz_ = zi - jp[3 * tb + 2];
              const double ra = fma(az, az, fma(ay, ay, ax * ax));
              const double rb = fma(bz_, bz_, fma(by_, by_, bx_ * bx_));
              mylist[64 * cnt] = (unsigned char)ta;
              cnt += (ta < mj && ra < rc2 && ta != self) ? 1 : 0;
              mylist[64 * cnt] = (unsigned char)tb;
              cnt += (tb < mj && rb < rc2 && tb != self) ? 1 : 0;
            }
            flush();
            if (kb >= mj) break;
          }
        }
      }
      acc_gather(acc, hc, NS);
      const bool lead = lane < hc;
      const CompDev &cd = md->comp[ci];
      double q[4] = {1.0, 0.0, 0.0, 0.0};
      int64_t orig = 0;
      if (lead) {
        orig = c.perm[hs + iloc];
        if (quat)
#pragma unroll
          for (int k = 0; k < 4; ++k) q[k] = quat[4 * (int64_t)(hs + iloc) + k];
        double dp[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < Acc::NSITE; ++a) dp[0] += acc.gs[a][0], dp[1] += acc.gs[a][1], dp[2] += acc.gs[a][2];
#pragma unroll
        for (int k = 0; k < 3; ++k) o.dpos[3 * orig + k] = o.gU * dp[k];
        if (o.dquat) {
          double dq[4] = {0.0, 0.0, 0.0, 0.0};
          if (quat) {
#pragma unroll
            for (int a = 0; a < SL; ++a)
              if (a < cd.n_lj) quat_vjp(q, cd.lj_pos[a], acc.gs[a], dq);
#pragma unroll
            for (int a = 0; a < SC; ++a)
              if (a < cd.n_chg) quat_vjp(q, cd.chg_pos[a], acc.gs[SL + a], dq);
#pragma unroll
            for (int a = 0; a < SD; ++a)
              if (a < cd.n_dip) {
                quat_vjp(q, cd.dip_pos[a], acc.gs[SL + SC + a], dq);
                quat_vjp(q, cd.dip_dir[a], acc.ga[a], dq);
              }
#pragma unroll
            for (int a = 0; a < SQ; ++a)
              if (a < cd.n_quad) {
                quat_vjp(q, cd.quad_pos[a], acc.gs[SL + SC + SD + a], dq);
                quat_vjp(q, cd.quad_dir[a], acc.ga[SD + a], dq);
              }
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) o.dquat[4 * orig + k] = o.gU * dq[k];
        }
      }
      if (PRM && o.pgrad) {
        // this molecule's parameter partials (zero on non-leading lanes), then per component a
        // fixed-order wave sum added to the block row under the ABI column of each slot
        double pv[PS::np];
        const double w = q[0], x = q[1], y = q[2], z = q[3];
        const double Am[3][3] = {{w * w + x * x - y * y - z * z, 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                                 {2.0 * (x * y + w * z), w * w - x * x + y * y - z * z, 2.0 * (y * z - w * x)},
                                 {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), w * w - x * x - y * y + z * z}};
        auto body = [&](const double *g, int k) { return Am[0][k] * g[0] + Am[1][k] * g[1] + Am[2][k] * g[2]; };
        const double on = lead ? 1.0 : 0.0;
#pragma unroll
        for (int a = 0; a < SL; ++a) {
          pv[5 * a] = on * acc.peps[a], pv[5 * a + 1] = on * acc.psig[a];
#pragma unroll
          for (int k = 0; k < 3; ++k) pv[5 * a + 2 + k] = on * body(acc.gs[a], k);
        }
#pragma unroll
        for (int a = 0; a < SC + SD + SQ; ++a) {
          pv[PS::chg + 4 * a] = on * acc.pmom[a];
#pragma unroll
          for (int k = 0; k < 3; ++k) pv[PS::chg + 4 * a + 1 + k] = on * body(acc.gs[SL + a], k);
        }
        const int ncomp = MIX ? md->ncomp : 1;
        for (int cc = 0; cc < ncomp; ++cc) {
          const CompDev &cdc = md->comp[cc];
          const double sel = (ci == cc) ? 1.0 : 0.0;
          const int base = md->param_off[cc];
#pragma unroll
          for (int a = 0; a < SL; ++a) {
            if (a < cdc.n_lj) {
#pragma unroll
              for (int k = 0; k < 5; ++k) {
                const double v = wave_sum(sel * pv[5 * a + k]);
                if (lane == 0) bsum[base + 5 * a + k] += o.gU * v;
              }
            }
          }
#pragma unroll
          for (int a = 0; a < SC + SD + SQ; ++a) {
            // kind and index of moment slot a in the compile-time layout
            const int kind = a < SC ? 0 : (a < SC + SD ? 1 : 2);
            const int ia = a - (kind == 0 ? 0 : (kind == 1 ? SC : SC + SD));
            const int nk = kind == 0 ? cdc.n_chg : (kind == 1 ? cdc.n_dip : cdc.n_quad);
            const int abi = 5 * cdc.n_lj + 4 * (kind == 0 ? ia : (kind == 1 ? cdc.n_chg + ia : cdc.n_chg + cdc.n_dip + ia));
            if (ia < nk) {
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const double v = wave_sum(sel * pv[PS::chg + 4 * a + k]);
                if (lane == 0) bsum[base + abi + k] += o.gU * v;
              }
            }
          }
        }
      }
    }
  }
  if (PRM && o.pgrad) {
    __syncthreads();
    double *row = o.pgrad + (int64_t)blockIdx.x * ncol;
    for (int k = tid; k < ncol; k += 64 * W) {
      double v = bsums[0][k];
      for (int w = 1; w < W; ++w) v += bsums[w][k];
      row[k] = v;
    }
  }
}

// Dense cells (mean occupancy >= 16) are shared by four wavefronts with windows of CAP molecules,
// sparser ones take one wavefront each with windows of CAP1 (smaller LDS per one-wave block).
template <typename R, int SL, int SC, int SD, int SQ, bool MIX, int CAP, int CAP1 = CAP>
int launch_adj(const CellsDev &cd, const md_model *m, const double *quat, const AdjOut &o, int64_t nb, double mean,
               hipStream_t s) {
  const bool prm = o.pgrad != nullptr;
  if (mean >= 16.0 && prm)
    k_adjoint<R, SL, SC, SD, SQ, MIX, CAP, 4, true><<<(unsigned)nb, 256, 0, s>>>(cd, m->dev, quat, m->host.rc2, o);
  else if (mean >= 16.0)
    k_adjoint<R, SL, SC, SD, SQ, MIX, CAP, 4, false><<<(unsigned)nb, 256, 0, s>>>(cd, m->dev, quat, m->host.rc2, o);
  else if (prm)
    k_adjoint<R, SL, SC, SD, SQ, MIX, CAP1, 1, true><<<(unsigned)nb, 64, 0, s>>>(cd, m->dev, quat, m->host.rc2, o);
  else
    k_adjoint<R, SL, SC, SD, SQ, MIX, CAP1, 1, false><<<(unsigned)nb, 64, 0, s>>>(cd, m->dev, quat, m->host.rc2, o);
  return check_hip(hipGetLastError(), "k_adjoint");
}

// Single-site LJ adjoint from one force evaluation (md_forces_adjoint): dpos = -gU F in place,
// and, when dparams is given, the parameter gradients with the same per-pair-end factors as the
// adjoint kernel (pe, ps, csh of the site pair) summed over both ends of every pair:
// gU (2 pe U, 2 ps (W / (4 eps) - P csh)), and the offset gradient sum_i dU/dr_i, which is zero
// (U does not change under a common translation; the single site sits at the centre).
__global__ __launch_bounds__(256) void k_lj_adjoint_finish(double *dpos, int64_t n3, double gU, const double *uw,
                                                           const int64_t *npairs, LJPair p, double *dparams) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) dpos[i] = -gU * dpos[i];
  if (dparams && i == 0) {
    dparams[0] = gU * (2.0 * p.pe * uw[0]);
    dparams[1] = gU * (2.0 * p.ps * (uw[1] / p.eps4 - (double)npairs[0] * p.csh));
    dparams[2] = dparams[3] = dparams[4] = 0.0;
  }
}

}  // namespace

int launch_lj_adjoint_finish(const md_model *m, double *dpos, int64_t N, double gU, const double *uw,
                             const int64_t *npairs, double *dparams, hipStream_t s) {
  k_lj_adjoint_finish<<<(unsigned)((3 * N + 255) / 256), 256, 0, s>>>(dpos, 3 * N, gU, uw, npairs,
                                                                     m->host.lj[0][0][0][0], dparams);
  return check_hip(hipGetLastError(), "k_lj_adjoint_finish");
}

CellsDev cells_dev(const md_cells *c);

int launch_adjoint(md_model *m, const md_cells *c, int precision, const AdjOut &o, const double *quat, hipStream_t s,
                   int64_t *nblocks) {
  const CellsDev cd = cells_dev(c);
  const int64_t nb = pair_blocks(c->ncell);
  *nblocks = nb;
  const bool f32 = precision == MD_FP32;
  const Shape &S = m->shape;
  const double mean = (double)c->N / (double)c->ncell;
  if (m->single_site)  // md_forces_adjoint takes these models through the force kernel
    return set_error(MD_EINVAL, "launch_adjoint: single-site model");
  if (m->fixed_shape && S.lj == 2 && S.chg == 0 && S.dip == 0 && S.quad == 1)
    return f32 ? launch_adj<float, 2, 0, 0, 1, false, 256, 64>(cd, m, quat, o, nb, mean, s)
               : launch_adj<double, 2, 0, 0, 1, false, 256, 64>(cd, m, quat, o, nb, mean, s);
  if (m->fixed_shape && S.lj == 3 && S.chg == 0 && S.dip == 1 && S.quad == 0)
    return f32 ? launch_adj<float, 3, 0, 1, 0, false, 256, 64>(cd, m, quat, o, nb, mean, s)
               : launch_adj<double, 3, 0, 1, 0, false, 256, 64>(cd, m, quat, o, nb, mean, s);
  return f32 ? launch_adj<float, MD_MAX_LJ, MD_MAX_CHG, MD_MAX_DIP, MD_MAX_QUAD, true, 64>(cd, m, quat, o, nb,
                                                                                                    mean, s)
             : launch_adj<double, MD_MAX_LJ, MD_MAX_CHG, MD_MAX_DIP, MD_MAX_QUAD, true, 64>(cd, m, quat, o, nb,
                                                                                                     mean, s);
}

}  // namespace mdcell
