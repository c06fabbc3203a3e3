// Kriging pass of the M-RA (Sec. 3.4, Prop. 2): posterior predictive mean
// and marginal variance of the latent process at prediction locations.
//
// In the whitened form of the forward kernels, for prediction rows S^P in
// leaf R with ancestors a_0..a_{M-1}:
//   U^^l  = (C_0(S^P, Q_{a_l}) - sum_{k<l} U^^k W^^k_{a_l}') L_{a_l}^{-T}      (row sweep)
//   L^M   = C_0(S^P, S_R) - sum_{k<M} U^^k W^^k_R'
//   E     = L^M L_Sigma^{-T}                  (so L^M Sigma^{-1} = E L_Sigma^{-1})
//   V^P   = sigma^2 - sum_k ||U^^k||^2        (diagonal)
//   B~^{M,k} = U^^k - E Y_k,  Y_k = L_Sigma^{-1} W^^k_R                (eq. bfrecursion, l = M)
//   for l = M-1..0 with Bh = B~^{l+1,l} Lt_{a_l}^{-T}:
//       mean += Bh z_w(a_l),  var += ||Bh||^2,
//       B~^{l,k} = B~^{l+1,k} - Bh Z_k(a_l),  k < l                    (eq. bfrecursion)
//   mean += E y_z,  var += V^P - ||E||^2,  y_z = L_Sigma^{-1} z
// where Lt_a Lt_a' = I + A^{l,l}_a is the whitened K~^{-1}, Z_k = Lt^{-1} A^{l,k}
// and z_w = Lt^{-1} w^l, all kept by the forward pass.
#include "common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace mra {

__device__ __forceinline__ double row_dot(const double* a, const double* b) {
  double s = 0.0;
  for (int j = 0; j < T; ++j) s += a[j] * b[j];
  return s;
}

// one 64-row prediction tile; with keep (MRA_JOINT) the whitened prior rows
// U^^k are also kept (off_pu) and the mean written in leaf order (off_pmean)
__global__ __launch_bounds__(NT) void k_predict(DevPlan P, const double* theta, double* mean, double* var, int keep,
                                                TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_SWEEP];
  __shared__ double mu[T], vv[T];
  const int64_t tk = tk0;
  const int32_t* task = P.pred_tasks + 2 * tk;
  const int leaf = task[0];
  const int64_t q0 = task[1];
  double* S = slice(P, 0);
  const CovP c = load_cov(theta, P.cov);
  const int M = P.M;
  const double* X = P.pred_xy + 2 * q0;
  const int nx = min(T, (int)(P.pleaf_n[leaf] - (q0 - P.pleaf_poff[leaf])));
  double* U = S + P.off_pw + q0 * T;      // plane l at U + l * ppad * T
  const int64_t pplane = P.ppad * T;
  row_sweep(P, S, c, X, nx, U, pplane, M, leaf, lds, lds + LDS_DOUBLES);
  if (keep) {
    for (int k = 0; k < M; ++k)
      for (int e = threadIdx.x; e < TT; e += NT) S[P.off_pu + (int64_t)k * pplane + q0 * T + e] = U[(int64_t)k * pplane + e];
  }
  // leaf quantities
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  const int nR = P.leaf_n[leaf];
  const double* Lsig = S + P.off_sig + P.leaf_soff[leaf] * TT;
  const double* dinv = S + P.off_dinv + P.leaf_doff[leaf] * TT;
  double* E = S + P.off_pl + tk * P.pl_stride;    // nb tiles: L^M, then E
  Acc acc;
  for (int jb = 0; jb < nb; ++jb) {
    const int64_t pj = poff + (int64_t)T * jb;
    acc_cov(acc, X, nx, P.obs_xy + 2 * pj, min(T, nR - T * jb), c, false, 0.0);
    // L^M_j, then E_j = (L^M_j - sum_{k<j} E_k L_{j,k}') L_jj^{-T}
    gemm_segs(acc, M + jb, [&](int q) {
      if (q < M) return seg<Op::N, Op::T>(U + (int64_t)q * pplane, T, S + P.off_wobs + (int64_t)q * P.plane + pj * T, T, -1.0);
      const int kb = q - M;
      return seg<Op::N, Op::T>(E + (int64_t)kb * TT, T, Lsig + ((int64_t)jb * nb + kb) * TT, T, -1.0);
    }, lds, round16(nx));
    acc_store(acc, E + (int64_t)jb * TT, T);
    __syncthreads();
    acc_zero(acc);
    gemm<Op::N, Op::T>(acc, E + (int64_t)jb * TT, T, dinv + (int64_t)jb * TT, T, T, 1.0, lds);
    acc_store(acc, E + (int64_t)jb * TT, T);
    __syncthreads();
  }
  // V^P, leaf mean and variance terms
  if (threadIdx.x < T) {
    const int r = threadIdx.x;
    double vp = c.s2;
    for (int k = 0; k < M; ++k) {
      const double* u = U + (int64_t)k * pplane + r * T;
      vp -= row_dot(u, u);
    }
    double m_leaf = 0.0, e2 = 0.0;
    const double* yz = S + P.off_y + (int64_t)M * P.plane;
    for (int jb = 0; jb < nb; ++jb) {
      const double* e = E + (int64_t)jb * TT + r * T;
      for (int j = 0; j < T; ++j) {
        m_leaf += e[j] * yz[(poff + (int64_t)T * jb + j) * T];
        e2 += e[j] * e[j];
      }
    }
    mu[r] = m_leaf;
    vv[r] = vp - e2;
  }
  __syncthreads();
  // B~^{M,k} = U^^k - E Y_k (in place over U^^k)
  for (int k = 0; k < M; ++k) {
    acc_load(acc, U + (int64_t)k * pplane, T);
    gemm_segs(acc, nb, [&](int jb) {
      return seg<Op::N, Op::N>(E + (int64_t)jb * TT, T, S + P.off_y + (int64_t)k * P.plane + (poff + (int64_t)T * jb) * T,
                               T, -1.0);
    }, lds, round16(nx));
    acc_store(acc, U + (int64_t)k * pplane, T);
  }
  __syncthreads();
  // up the tree: eq. bfrecursion and the weight terms of eq. prediction
  for (int l = M - 1; l >= 0; --l) {
    const int64_t al = ancestor(P, M, leaf, l);
    double* Bl = U + (int64_t)l * pplane;
    if (!post_active(P, l, al)) {
      // no observation below a_l: its posterior is its prior (Lt = I, Z = 0,
      // z_w = 0), so Bh = B~^{l+1,l} and only the variance term remains
      if (threadIdx.x < T) {
        const double* b = Bl + threadIdx.x * T;
        vv[threadIdx.x] += row_dot(b, b);
      }
      __syncthreads();
      continue;
    }
    Post po = post_of(P, S, l, al);
    acc_zero(acc);
    gemm<Op::N, Op::T>(acc, Bl, T, po.Lti(), T, T, 1.0, lds);   // Bh = B~^{l+1,l} Lt^{-T}
    acc_store(acc, Bl, T);
    __syncthreads();
    if (threadIdx.x < T) {
      const double* b = Bl + threadIdx.x * T;
      mu[threadIdx.x] += row_dot(b, po.zw());
      vv[threadIdx.x] += row_dot(b, b);
    }
    for (int k = 0; k < l; ++k) {
      double* Bk = U + (int64_t)k * pplane;
      acc_load(acc, Bk, T);
      gemm<Op::N, Op::N>(acc, Bl, T, po.Z(k), T, T, -1.0, lds);
      acc_store(acc, Bk, T);
    }
    __syncthreads();
  }
  if (threadIdx.x < T) {
    const int64_t g = P.pred_gidx[q0 + threadIdx.x];
    if (g >= 0) {
      mean[g] = mu[threadIdx.x];
      var[g] = vv[threadIdx.x];
    }
    if (keep) S[P.off_pmean + q0 + threadIdx.x] = g >= 0 ? mu[threadIdx.x] : 0.0;
  }
}

// after the forward pass; with MRA_CHECKPOINT the leaf planes W^ and Y of
// each chunk are recomputed (from y) before its prediction tiles
hipError_t launch_predict(const mra_plan_s& H, const double* y, const double* theta, double* mean, double* var,
                          hipStream_t st, bool keep) {
  const int kp = keep ? 1 : 0;
  const int64_t npt = (int64_t)H.pred_tasks.size() / 2;
  if (H.nchunks > 1) {
    for (int c = 0; c < H.nchunks; ++c) {
      const int64_t t0 = H.ck_pred[c], t1 = H.ck_pred[c + 1];
      if (t1 <= t0) continue;
      const hipError_t e = launch_leaf_planes(H, c, y, theta, 1, st, 0, false);
      if (e != hipSuccess) return e;
      const DevPlan P = chunk_plan(H, c);
      Runner run{P, 1, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
      run.tuned(F_PREDICT, MAP_CHUNKED, "predict", -1, npt ? H.pf.predict * (double)(t1 - t0) / (double)npt : 0.0,
                1, nullptr, k_predict, t0, t1, theta, mean, var, kp);
    }
    return hipGetLastError();
  }
  const DevPlan& P = H.dp;
  Runner run{P, 1, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  run.tuned(F_PREDICT, MAP_CHUNKED, "predict", -1, H.pf.predict, 1, nullptr, k_predict, 0, npt, theta, mean, var, kp);
  return hipGetLastError();
}

}  // namespace mra
