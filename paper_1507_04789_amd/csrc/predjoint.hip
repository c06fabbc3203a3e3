// Joint posterior predictive distribution of the latent process at the
// prediction locations (Prop. 2 and the remark after it): covariance matrix
// and conditional simulation.
//
// By Prop. 2 the posterior predictive has the M-RA form
//   y_M(S^P_R) | z = sum_{m<M} B~^{m+1,m}_R eta~_{a_m} + delta~_R,
// with independent weights eta~_{a_m} ~ N(K~ w^m, K~) per region and an
// independent remainder delta~_R ~ N(L^M Sigma^{-1} z_R, V^P - L^M Sigma^{-1} L^M')
// per leaf.  In the whitened form of the kriging pass, K~_{a_m} = Lt^{-T} Lt^{-1}
// at every region (Lt = I where no observation lies below), so with the
// factor rows Bh^m = B~^{m+1,m} Lt_{a_m}^{-T} that k_predict leaves in its
// prediction planes,
//   Psi(s, s') = sum over the levels m < M whose region contains both
//                points of Bh^m(s) . Bh^m(s')
//              + [same leaf] (C_0(s, s') - sum_{k<M} U^^k(s) . U^^k(s') - E(s) . E(s')),
// where U^^k are the whitened prior rows of the points (V^P = C_0 -
// sum_k U^^k U^^k') and E = L^M L_Sigma^{-T} (L^M Sigma^{-1} L^M' = E E').
// A conditional draw with standard normals xi is
//   mean + sum_m Bh^m xi_{a_m} + chol(remainder block of the leaf) xi_R.
#include "common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace mra {

namespace {

// the 64 prediction rows of prediction task t
struct PTile {
  int leaf;
  int64_t q0;
  int nx;
  int bi;    // tile index within the leaf
  int nbp;   // tiles of the leaf
};
__device__ __forceinline__ PTile ptile(const DevPlan& P, int64_t t) {
  PTile p;
  p.leaf = P.pred_tasks[2 * t];
  p.q0 = P.pred_tasks[2 * t + 1];
  const int64_t po = P.pleaf_poff[p.leaf];
  p.nx = min(T, (int)(P.pleaf_n[p.leaf] - (p.q0 - po)));
  p.bi = (int)((p.q0 - po) / T);
  p.nbp = (int)((P.pleaf_poff[p.leaf + 1] - po) / T);
  return p;
}

// deepest level below M at which two leaves share their region (-1: none)
__device__ __forceinline__ int shared_levels(const DevPlan& P, int li, int lj) {
  int m = -1;
  for (int l = 0; l < P.M; ++l)
    if (ancestor(P, P.M, li, l) == ancestor(P, P.M, lj, l)) m = l;
    else break;
  return m;
}

// covariance tile of prediction tiles (a, b): with weights the region terms
// sum_m Bh^m_a Bh^m_b'; for tiles of one leaf the remainder block
// C_0 - sum_k U^^k_a U^^k_b' - E_a E_b'
__device__ void pcov_tile(const DevPlan& P, double* S, const CovP& c, const PTile& a, int64_t ta, const PTile& b,
                          int64_t tb, bool weights, Acc& acc, double* lds) {
  const int M = P.M;
  const int64_t pplane = P.ppad * T;
  const bool same = a.leaf == b.leaf;
  const int mw = weights ? (same ? M - 1 : shared_levels(P, a.leaf, b.leaf)) : -1;
  const int nbo = same ? (int)((P.leaf_poff[a.leaf + 1] - P.leaf_poff[a.leaf]) / T) : 0;
  if (same) acc_cov(acc, P.pred_xy + 2 * a.q0, a.nx, P.pred_xy + 2 * b.q0, b.nx, c, ta == tb, 0.0);
  else acc_zero(acc);
  const double* E = S + P.off_pl;
  const int nseg = (mw + 1) + (same ? M + nbo : 0);
  gemm_segs2(acc, nseg, [&](int q) {
    if (q <= mw)
      return seg<Op::N, Op::T>(S + P.off_pw + (int64_t)q * pplane + a.q0 * T, T,
                               S + P.off_pw + (int64_t)q * pplane + b.q0 * T, T, 1.0);
    q -= mw + 1;
    if (q < M)
      return seg<Op::N, Op::T>(S + P.off_pu + (int64_t)q * pplane + a.q0 * T, T,
                               S + P.off_pu + (int64_t)q * pplane + b.q0 * T, T, -1.0);
    q -= M;
    return seg<Op::N, Op::T>(E + ta * P.pl_stride + (int64_t)q * TT, T, E + tb * P.pl_stride + (int64_t)q * TT, T,
                             -1.0);
  }, lds, round16(a.nx), round16(b.nx));
}

}  // namespace

// dense covariance: task t -> tile pair (a, b), a >= b, of the prediction
// tiles; written to cov[n_pred][n_pred] in the caller's order (both triangles)
__global__ __launch_bounds__(NT) void k_pcov(DevPlan P, const double* theta, double* cov, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  int64_t ta = (int64_t)((sqrt(8.0 * (double)tk0 + 1.0) - 1.0) * 0.5);
  while (ta * (ta + 1) / 2 > tk0) --ta;
  while ((ta + 1) * (ta + 2) / 2 <= tk0) ++ta;
  const int64_t tb = tk0 - ta * (ta + 1) / 2;
  double* S = slice(P, 0);
  const CovP c = load_cov(theta, P.cov);
  const PTile a = ptile(P, ta), b = ptile(P, tb);
  Acc acc;
  pcov_tile(P, S, c, a, ta, b, tb, true, acc, lds);
  const int64_t np = P.n_pred;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = acc_row(bi, v), j = acc_col(bj);
        const int64_t gi = P.pred_gidx[a.q0 + i], gj = P.pred_gidx[b.q0 + j];
        if (gi < 0 || gj < 0) continue;
        cov[gi * np + gj] = acc.c[bi][bj][v];
        if (ta != tb) cov[gj * np + gi] = acc.c[bi][bj][v];
      }
}

// remainder block of a leaf's prediction points, tile (bi, bj), bi >= bj
__global__ __launch_bounds__(NT) void k_pcd(DevPlan P, const double* theta, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int leaf = P.pcd_tasks[3 * tk0], bi = P.pcd_tasks[3 * tk0 + 1], bj = P.pcd_tasks[3 * tk0 + 2];
  double* S = slice(P, 0);
  const CovP c = load_cov(theta, P.cov);
  // prediction task indices of the two tiles: tasks are in leaf order with
  // consecutive tiles per leaf, the first located by a binary search
  int64_t lo = 0, hi = P.ppad / T;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (P.pred_tasks[2 * mid] < leaf) lo = mid + 1;
    else hi = mid;
  }
  const int64_t ta = lo + bi, tb = lo + bj;
  const PTile a = ptile(P, ta), b = ptile(P, tb);
  Acc acc;
  pcov_tile(P, S, c, a, ta, b, tb, false, acc, lds);
  const int nbp = a.nbp;
  acc_store(acc, S + P.off_pcd + (P.pleaf_soff[leaf] + (int64_t)bi * nbp + bj) * TT, T);
}

// Cholesky of each leaf's remainder block
__global__ __launch_bounds__(NT, 2) void k_pred_potrf(DevPlan P, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  __shared__ double lds_x[T * PLD];
  __shared__ double red[8];
  const int leaf = P.pfac_tasks[tk0];
  double* S = slice(P, 0);
  const int nbp = (int)((P.pleaf_poff[leaf + 1] - P.pleaf_poff[leaf]) / T);
  bool ok = true;
  (void)potrf_tiles(S + P.off_pcd + P.pleaf_soff[leaf] * TT, S + P.off_pdinv + P.pleaf_doff[leaf] * TT, nbp,
                    P.pleaf_n[leaf], lds, lds_x, red, ok);
  if (threadIdx.x == 0 && !ok) record_failure(P, S, P.M, leaf);
}

// standard normals of draw d < nd into the padded work rows: the region
// weights as given, the remainder ones moved to leaf order; rows and entries
// past the draws and the points are zero
__global__ void k_sim_gather(DevPlan P, const double* eps, int64_t n_eps, int nd) {
  double* S = slice(P, 0);
  const int64_t nreg = P.reg_base[P.M] * T;
  const int d = blockIdx.y;
  double* row = S + P.off_sim + (int64_t)d * P.n_sim;
  const double* src = eps + (int64_t)d * n_eps;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < P.n_sim; e += (int64_t)gridDim.x * NT) {
    double v = 0.0;
    if (d < nd) {
      if (e < nreg) v = src[e];
      else {
        const int64_t g = P.pred_gidx[e - nreg];
        v = g >= 0 ? src[nreg + g] : 0.0;
      }
    }
    row[e] = v;
  }
}

// draws of one prediction tile, 64 draws as the columns of a tile:
// mean + sum_m Bh^m xi_{a_m} + sum_{jb <= bi} Lrem_{bi, jb} xi_{leaf, jb}
__global__ __launch_bounds__(NT) void k_sim(DevPlan P, double* out, int nd, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  double* S = slice(P, 0);
  const PTile a = ptile(P, tk0);
  const int M = P.M;
  const int64_t pplane = P.ppad * T;
  const double* xi = S + P.off_sim;
  const int64_t nreg = P.reg_base[M] * T;
  const double* Lr = S + P.off_pcd + P.pleaf_soff[a.leaf] * TT;
  Acc acc;
  acc_zero(acc);
  gemm_segs2(acc, M + a.bi + 1, [&](int q) {
    if (q < M) {
      const int64_t reg = P.reg_base[q] + ancestor(P, M, a.leaf, q);
      return seg<Op::N, Op::T>(S + P.off_pw + (int64_t)q * pplane + a.q0 * T, T, xi + reg * T, P.n_sim, 1.0);
    }
    const int jb = q - M;
    return seg<Op::N, Op::T>(Lr + ((int64_t)a.bi * a.nbp + jb) * TT, T,
                             xi + nreg + P.pleaf_poff[a.leaf] + (int64_t)jb * T, P.n_sim, 1.0);
  }, lds, round16(a.nx), round16(nd));
  const double* mu = S + P.off_pmean;
  const int64_t np = P.n_pred;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = acc_row(bi, v), d = acc_col(bj);
        const int64_t g = P.pred_gidx[a.q0 + i];
        if (g >= 0 && d < nd) out[(int64_t)d * np + g] = mu[a.q0 + i] + acc.c[bi][bj][v];
      }
}

// after the forward pass and a kriging pass that kept its rows
hipError_t launch_predict_cov(const mra_plan_s& H, const double* theta, double* cov, hipStream_t st) {
  const DevPlan& P = H.dp;
  Runner run{P, 1, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  const int64_t nt = (int64_t)H.pred_tasks.size() / 2;
  run("pred_cov", -1, 0.0, k_pcov, nt * (nt + 1) / 2, theta, cov);
  return hipGetLastError();
}

hipError_t launch_simulate(const mra_plan_s& H, const double* theta, const double* eps, int64_t n_eps, int nd,
                           double* out, hipStream_t st) {
  const DevPlan& P = H.dp;
  Runner run{P, 1, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  run("pred_rem", -1, 0.0, k_pcd, (int64_t)H.pcd_tasks.size() / 3, theta);
  run("pred_potrf", -1, 0.0, k_pred_potrf, (int64_t)H.pfac_tasks.size());
  int64_t gx = (P.n_sim + NT - 1) / NT;
  if (gx > 2048) gx = 2048;
  hipLaunchKernelGGL(k_sim_gather, dim3((unsigned)gx, SIM_DRAWS), dim3(NT), 0, st, P, eps, n_eps, nd);
  run("simulate", -1, 0.0, k_sim, (int64_t)H.pred_tasks.size() / 2, out, nd);
  return hipGetLastError();
}

}  // namespace mra
