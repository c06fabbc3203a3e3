// Reverse pass of the M-RA log-likelihood: d loglik / d(log sigma^2,
// log kappa, log tau^2), hand-written adjoint of the forward kernels.
//
// Every posterior step (a region's, and the leaves' definitions) has the
// form F = X' P^{-1} X, d += log|P|, with X = [A^{m,<m} | w^m] and
// P = I + A^{m,m} (whitened K~^{-1}) at a region, X = [W^_R | z_R] and
// P = Sigma_R at a leaf; the outputs are A~ = A - F_AA, w~ = w - F_Aw and
// u -= F_ww.  With the cotangent Fbar of F (symmetric) and dbar = -1/2,
//   Xbar = 2 P^{-1} X Fbar = 2 V Fbar,  Pbar = -V Fbar V' - 1/2 P^{-1},
// V = P^{-1} X = L^{-T} (L^{-1} X), which only needs the stored factors.
// At a region the outputs are A - F_AA, w - F_Aw and u - F_ww, so
// Fbar = [[-S, -wbar/2], [-wbar'/2, 1/2]]; at a leaf they are F itself
// (A~ = F_AA, w~ = F_Az, u = F_zz), so Fbar = [[S, wbar/2], [wbar'/2, -1/2]].
// S is the symmetric form of the cotangent of the parent's A (off-diagonal
// blocks halved); every region inherits its parent's cotangents for the
// blocks k, l < m, so the cotangent of A^{k,l} below region a_k is the one
// stored at a_k (row k).
//
// The prior recursion (eq. priorw, whitened) is reversed row by row:
// W^^l = W^l L_{a_l}^{-T} gives Wbar^l = W^^bar^l L_{a_l}^{-1} and
// L_{a_l}-bar = -tril(sum_rows Wbar^l' W^^l); the ancestors' cotangents are
// subtree sums Tsum^{l,k} = sum over rows of Wbar^l' W^^k, accumulated with
// the child sums of the tree (no atomics); L_R = chol(W^m_R) is reversed by
// the Cholesky adjoint Wbar^m = sym(L^{-T} Phi(L' Lbar) L^{-1}).  Every
// covariance entry's cotangent Cbar is contracted with dC/dlog sigma^2 = C
// and dC/dlog kappa; dloglik/dlog tau^2 = tau^2 tr(Sigma-bar) over the leaves.
#include "common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace mra {

// segment alpha * V * S^{k,c}, S from the cotangents stored at the
// ancestors a_k, a_c of a region at level `lev`, index `idx`
__device__ __forceinline__ Seg seg_S(const DevPlan& P, double* S, const double* V, int k, int c, int lev,
                                     int64_t idx, double alpha) {
  if (k > c) return seg<Op::N, Op::N>(V, T, grad_of(P, S, k, ancestor(P, lev, idx, k)).G(c), T, 0.5 * alpha);
  if (k < c) return seg<Op::N, Op::T>(V, T, grad_of(P, S, c, ancestor(P, lev, idx, c)).G(k), T, 0.5 * alpha);
  return seg<Op::N, Op::N>(V, T, grad_of(P, S, k, ancestor(P, lev, idx, k)).G(k), T, alpha);
}

__device__ __forceinline__ const double* wbar_omega_of(const DevPlan& P, double* S, int k, int lev, int64_t idx) {
  return grad_of(P, S, k, ancestor(P, lev, idx, k)).wbar_omega();
}

__device__ void write_partial(const DevPlan& P, double* S, int64_t slot, double g[3], double* red) {
  double a = block_sum(g[0], red);
  double b = block_sum(g[1], red);
  double c = block_sum(g[2], red);
  if (threadIdx.x == 0) {
    double* o = S + P.off_gpart + slot * 4;
    o[0] = a;
    o[1] = b;
    o[2] = c;
    o[3] = 0.0;
  }
}

// ---------------------------------------------------------------- posterior
// region (m, i), top-down: G^{m,l} = Xbar_l, G^{m,m} = Pbar, wbar^m = xbar_w
__global__ __launch_bounds__(NT, 4) void k_rpost(DevPlan P, int m, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int th = blockIdx.y;
  const int64_t i = P.act_post[P.act_post_off[m] + tk0];
  double* S = slice(P, th);
  Post po = post_of(P, S, m, i);
  Grad gr = grad_of(P, S, m, i);
  double* vw = gr.scratch();          // v_w = Lt^{-T} z_w (first T entries of the scratch tile)
  Acc acc;
  for (int l = 0; l < m; ++l) {       // V_l = Lt^{-T} Z_l, kept in the Tsum tiles (free until later)
    acc_zero(acc);
    gemm<Op::T, Op::N>(acc, po.Lti(), T, po.Z(l), T, T, 1.0, lds);
    acc_store(acc, gr.Tsum(0, 0) + (int64_t)l * TT, T);
  }
  if (threadIdx.x < T) {
    // q from threadIdx.x up; each batch of 16 rows is loaded before it is used
    double s = 0.0;
    const double* Li = po.Lti();
    const double* zw = po.zw();
    for (int q0 = 0; q0 < T; q0 += 16) {
      if (q0 + 15 < (int)threadIdx.x) continue;
      double lv[16], zv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        lv[j] = Li[(q0 + j) * T + threadIdx.x];
        zv[j] = zw[q0 + j];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (q0 + j >= (int)threadIdx.x) s += lv[j] * zv[j];
    }
    vw[threadIdx.x] = s;
  }
  __syncthreads();
  const double* V0 = gr.Tsum(0, 0);
  for (int l = 0; l < m; ++l) {       // Xbar_l = -2 sum_k V_k S^{k,l} - v_w wbar^l'
    acc_zero(acc);
    gemm_segs2(acc, m, [&](int k) { return seg_S(P, S, V0 + (int64_t)k * TT, k, l, m, i, -2.0); }, lds);
    const double* wb = wbar_omega_of(P, S, l, m, i);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc.c[bi][bj][v] -= vw[acc_row(bi, v)] * wb[acc_col(bj)];
    acc_store(acc, gr.G(l), T);
  }
  {                                   // xbar_w = -sum_k V_k wbar^k + v_w, four threads per row
    const int r = threadIdx.x >> 2, part = threadIdx.x & 3;
    double s = 0.0;
    for (int k = 0; k < m; ++k) {
      const double* Vk = V0 + (int64_t)k * TT + r * T + part * 16;
      const double* wb = wbar_omega_of(P, S, k, m, i) + part * 16;
#pragma unroll
      for (int j = 0; j < 16; ++j) s += Vk[j] * wb[j];
    }
    s = quad_sum(s);
    if (part == 0) gr.wbar_omega()[r] = vw[r] - s;
  }
  __syncthreads();
  // Pbar = -1/2 (sum_l Xbar_l V_l' + xbar_w v_w' + Lt^{-T} Lt^{-1})
  acc_zero(acc);
  gemm_segs2(acc, m + 1, [&](int l) {
    if (l < m) return seg<Op::N, Op::T>(gr.G(l), T, V0 + (int64_t)l * TT, T, -0.5);
    return seg<Op::T, Op::N>(po.Lti(), T, po.Lti(), T, -0.5);
  }, lds);
  const double* xw = gr.wbar_omega();
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc.c[bi][bj][v] -= 0.5 * xw[acc_row(bi, v)] * vw[acc_col(bj)];
  // G(m) = sym(Pbar), the transpose read from LDS
  acc_to_lds(acc, lds);
  __syncthreads();
  double* Gm = gr.G(m);
#pragma unroll
  for (int q = 0; q < TT / NT; ++q) {
    const int e = threadIdx.x + q * NT, r = e >> 6, cc = e & 63;
    Gm[e] = 0.5 * (lds[r * PLD + cc] + lds[cc * PLD + r]);
  }
}

// ---------------------------------------------------------------- leaves
// V = L_Sigma^{-T} Y for one column plane (backward substitution by tiles).
// After the updates the right-hand side tile stays in LDS for the product
// with the diagonal inverse instead of a round trip through global memory
// (same products in the same order).
__global__ __launch_bounds__(NT, 4) void k_rleaf_v(DevPlan P, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_SWEEP];
  const int th = blockIdx.y;
  const int32_t* task = P.trsm_tasks + 2 * tk0;
  const int leaf = task[0], cpl = task[1];
  double* S = slice(P, th);
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  const double* base = S + P.off_sig + P.leaf_soff[leaf] * TT;
  const double* dinv = S + P.off_dinv + P.leaf_doff[leaf] * TT;
  const double* Y = S + P.off_y + cpl * P.plane + poff * T;
  double* V = S + P.off_v + cpl * P.plane + poff * T;
  const int nR = P.leaf_n[leaf];
  // the reverse pass reads only column 0 of the data plane's V (the data
  // plane's other columns are zero or, after a trend fit, cleared)
  const int nc = cpl == P.M ? 16 : T;
  Acc acc;
  for (int ib = nb - 1; ib >= 0; --ib) {
    const int mr = round16(min(T, nR - T * ib));
    const double* R = Y + (int64_t)ib * TT;   // right-hand side
    if (ib < nb - 1) {                         // updated by the tiles below, then kept in LDS
      acc_load(acc, R, T);
      gemm_segs2(acc, nb - 1 - ib, [&](int q) {
        const int jb = ib + 1 + q;
        return seg<Op::T, Op::N>(base + ((int64_t)jb * nb + ib) * TT, T, V + (int64_t)jb * TT, T, -1.0);
      }, lds, mr, nc);
      acc_to_lds(acc, lds);
      __syncthreads();
      acc_zero(acc);
      gemm_lds_b(acc, dinv + (int64_t)ib * TT, T, true, lds, 1.0, lds + LDS_DOUBLES, mr, nc);
    } else {
      acc_zero(acc);
      gemm_segs(acc, 1, [&](int) { return seg<Op::T, Op::N>(dinv + (int64_t)ib * TT, T, R, T, 1.0); }, lds, mr, nc);
    }
    acc_store(acc, V + (int64_t)ib * TT, T);
    __syncthreads();
  }
}

// tile column j < nb - 1 of L_Sigma^{-1} below the diagonal (forward
// substitution of the identity); the diagonal tiles are the inverses the
// factorisation keeps, read in place.  Each new tile stays in LDS for its
// product with the diagonal inverse (same products in the same order as a
// store and reload).
__global__ __launch_bounds__(NT, 3) void k_rleaf_linv(DevPlan P, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_SWEEP];
  const int th = blockIdx.y;
  const int32_t* task = P.linv_tasks + 2 * tk0;
  const int leaf = task[0], j = task[1];
  double* S = slice(P, th);
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  const double* base = S + P.off_sig + P.leaf_soff[leaf] * TT;
  const double* dinv = S + P.off_dinv + P.leaf_doff[leaf] * TT;
  double* Li = S + P.off_linv + P.leaf_soff[leaf] * TT;
  Acc acc;
  for (int ib = j + 1; ib < nb; ++ib) {
    acc_zero(acc);
    gemm_segs(acc, ib - j, [&](int q) {
      const int kb = j + q;
      const double* Xkj = kb == j ? dinv + (int64_t)j * TT : Li + ((int64_t)kb * nb + j) * TT;
      return seg<Op::N, Op::N>(base + ((int64_t)ib * nb + kb) * TT, T, Xkj, T, -1.0);
    }, lds);
    acc_to_lds(acc, lds);
    __syncthreads();
    acc_zero(acc);
    gemm_lds_b(acc, dinv + (int64_t)ib * TT, T, false, lds, 1.0, lds + LDS_DOUBLES);
    acc_store(acc, Li + ((int64_t)ib * nb + j) * TT, T);
    __syncthreads();
  }
}

// Q = V Fbar for one 64-row tile and one column plane c (c = M: the z column)
__global__ __launch_bounds__(NT) void k_rleaf_q(DevPlan P, double* grad_y, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int th = blockIdx.y;
  const int M = P.M;
  const int64_t gid = tk0;
  const int64_t tsk = gid / (M + 1);
  const int c = (int)(gid % (M + 1));
  const int32_t* task = P.row_tasks + 2 * tsk;
  const int leaf = task[0];
  const int64_t p0 = task[1];
  double* S = slice(P, th);
  const double* V = S + P.off_v + p0 * T;
  const double* vz = S + P.off_v + (int64_t)M * P.plane + p0 * T;   // column 0
  double* Q = S + P.off_q + (int64_t)c * P.plane + p0 * T;
  if (c < M) {
    Acc acc;
    acc_zero(acc);
    const int nx = min(T, (int)(P.leaf_n[leaf] - (p0 - P.leaf_poff[leaf])));
    gemm_segs2(acc, M, [&](int k) { return seg_S(P, S, V + (int64_t)k * P.plane, k, c, M, leaf, 1.0); }, lds,
              round16(nx));
    const double* wb = wbar_omega_of(P, S, c, M, leaf);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc.c[bi][bj][v] += 0.5 * vz[acc_row(bi, v) * T] * wb[acc_col(bj)];
    acc_store(acc, Q, T);
  } else {
    // q_z = 1/2 sum_k V_k wbar^k - 1/2 v_z in column 0, zero elsewhere;
    // four threads per row, each over a quarter of the columns
    const int r = threadIdx.x >> 2, part = threadIdx.x & 3;
    double s = 0.0;
    for (int k = 0; k < M; ++k) {
      const double* Vk = V + (int64_t)k * P.plane + r * T + part * 16;
      const double* wb = wbar_omega_of(P, S, k, M, leaf) + part * 16;
#pragma unroll
      for (int j = 0; j < 16; ++j) s += Vk[j] * wb[j];
    }
    s = quad_sum(s);
    double* qr = Q + r * T + part * 16;
#pragma unroll
    for (int j = 0; j < 16; ++j) qr[j] = 0.0;
    if (part == 0) {
      qr[0] = 0.5 * s - 0.5 * vz[r * T];
      // the data gradient is the z column of Xbar = 2 V Fbar: sum_k V_k wbar^k - v_z
      if (grad_y) {
        const int64_t g = P.obs_gidx[p0 + r];
        if (g >= 0) grad_y[(int64_t)th * P.n + g] = s - vz[r * T];
      }
    }
  }
}

// Sigma-bar tile (bi, bj) = -sum_c Q_c[bi] V_c[bj]' - 1/2 (Sigma^{-1})_{bi,bj},
// contracted with the leaf covariance tile
__global__ __launch_bounds__(NT) void k_rleaf_sbar(DevPlan P, const double* theta, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  __shared__ double red[8];
  const int th = blockIdx.y;
  const int64_t tk = tk0;
  const int32_t* task = P.sig_tasks + 3 * tk;
  const int leaf = task[0], bi = task[1], bj = task[2];
  double* S = slice(P, th);
  const CovP cp = load_cov(theta + 3 * th, P.cov);
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  const int nR = P.leaf_n[leaf];
  const int64_t pi = poff + (int64_t)T * bi, pj = poff + (int64_t)T * bj;
  const double* Li = S + P.off_linv + P.leaf_soff[leaf] * TT;
  const double* dinv = S + P.off_dinv + P.leaf_doff[leaf] * TT;
  // tile (r, c) of L^{-1}: the diagonal ones are the factorisation's inverses
  auto li = [&](int r, int c) { return r == c ? dinv + (int64_t)r * TT : Li + ((int64_t)r * nb + c) * TT; };
  const int nvi = min(T, nR - T * bi), nvj = min(T, nR - T * bj);
  Acc acc;
  acc_zero(acc);
  gemm_segs2(acc, P.M + 1 + (nb - bi), [&](int q) {
    // Q of the data plane is zero outside column 0: K = 16 covers it
    if (q <= P.M)
      return seg<Op::N, Op::T>(S + P.off_q + q * P.plane + pi * T, T, S + P.off_v + q * P.plane + pj * T, T, -1.0,
                               q == P.M ? 1 : T / KC);
    const int kb = bi + q - (P.M + 1);
    return seg<Op::T, Op::N>(li(kb, bi), T, li(kb, bj), T, -0.5);
  }, lds, round16(nvi), round16(nvj));
  double* out = S + P.off_sbar + (P.leaf_soff[leaf] + (int64_t)bi * nb + bj) * TT;
  if (bi == bj) {      // a diagonal tile is symmetrised, the transpose read from LDS
    acc_to_lds(acc, lds);
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = acc_row(a, v), q = acc_col(b);
          acc.c[a][b][v] = 0.5 * (lds[r * PLD + q] + lds[q * PLD + r]);
        }
  }
  acc_store(acc, out, T);
  double g[3] = {0.0, 0.0, 0.0};
  acc_cov_contract(acc, P.obs_xy + 2 * pi, nvi, P.obs_xy + 2 * pj, nvj, cp, bi == bj, g);
  const double wgt = (bi == bj) ? 1.0 : 2.0;   // lower tiles stand for both triangles
  g[0] *= wgt;
  g[1] *= wgt;
  write_partial(P, S, P.leaf_soff[leaf] + (int64_t)bi * nb + bj, g, red);
}

// Reverse row sweep for 64 rows (points X, nx valid) of a region at level
// lev, left-looking: for l = lev-1..0,
//   W^-bar^l = init_l + extra_l - sum_{l' > l} Wbar^{l'} W^^l_{a_{l'}},
//   Wbar^l = W^-bar^l L_{a_l}^{-1}, contracted with C_0(X, Q_{a_l}),
// where init(acc, l) loads the cotangent of W^^l from outside the prior
// recursion and extra(l, q), q < nextra, adds further product segments to
// it.  rows + l*bstride receive Wbar^l.
template <class Init, class Extra>
__device__ void row_sweep_reverse(const DevPlan& P, double* S, const CovP& c, const double* X, int nx, double* rows,
                                  int64_t bstride, int lev, int64_t idx, double g[3], double* lds, Init init,
                                  int nextra, Extra extra) {
  Acc acc;
  const int mr = round16(nx);
  for (int l = lev - 1; l >= 0; --l) {
    const int64_t al = ancestor(P, lev, idx, l);
    const double* Pa = prior_reg(P, S, l, al);
    double* Rl = rows + l * bstride;
    init(acc, l);
    gemm_segs2(acc, nextra + lev - 1 - l, [&](int q) {
      if (q < nextra) return extra(l, q);
      const int lp = l + 1 + (q - nextra);
      return seg<Op::N, Op::N>(rows + lp * bstride, T, prior_reg(P, S, lp, ancestor(P, lev, idx, lp)) + (int64_t)l * TT,
                               T, -1.0);
    }, lds, mr);
    // W-bar^l = W^-bar^l L^{-1}: the left factor stays in LDS
    acc_to_lds(acc, lds);
    __syncthreads();
    acc_zero(acc);
    gemm_lds_a(acc, lds, Pa + (l + 1) * TT, T, true, 1.0, lds + LDS_DOUBLES, mr);
    acc_cov_contract(acc, X, nx, knots_of(P, l, al), P.rl[l], c, false, g);
    acc_store(acc, Rl, T);
    __syncthreads();
  }
}

// leaf rows: the cotangent of W^_R from the leaf step is 2 Q - 2 Sigma-bar W^_R
// (computed here as the first product segments), then the reverse sweep
__global__ __launch_bounds__(NT, 3) void k_rrows_leaf(DevPlan P, const double* theta, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_SWEEP];
  __shared__ double red[8];
  const int th = blockIdx.y;
  const int64_t tk = tk0;
  const int32_t* task = P.row_tasks + 2 * tk;
  const int leaf = task[0];
  const int64_t p0 = task[1];
  double* S = slice(P, th);
  const CovP c = load_cov(theta + 3 * th, P.cov);
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  const int bi = (int)((p0 - poff) / T);
  const int nx = min(T, (int)(P.leaf_n[leaf] - (p0 - poff)));
  const double* Sb = S + P.off_sbar + P.leaf_soff[leaf] * TT;
  double g[3] = {0.0, 0.0, 0.0};
  auto init = [&](Acc& acc, int l) {
    acc_load(acc, S + P.off_q + (int64_t)l * P.plane + p0 * T, T);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc.c[a][b] *= 2.0;
  };
  auto extra = [&](int l, int bj) {
    const double* W = S + P.off_wobs + (int64_t)l * P.plane + (poff + (int64_t)bj * T) * T;
    if (bj <= bi) return seg<Op::N, Op::N>(Sb + ((int64_t)bi * nb + bj) * TT, T, W, T, -2.0);
    return seg<Op::T, Op::N>(Sb + ((int64_t)bj * nb + bi) * TT, T, W, T, -2.0);
  };
  row_sweep_reverse(P, S, c, P.obs_xy + 2 * p0, nx, S + P.off_wbar + p0 * T, P.plane, P.M, leaf, g, lds, init, nb,
                    extra);
  write_partial(P, S, P.n_sig_tiles + tk, g, red);
}

// Tsum^{l,k} of a level-(M-1) region: sum over its leaves' rows of Wbar^l' W^^k
__global__ __launch_bounds__(NT) void k_rT_leaf(DevPlan P, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int th = blockIdx.y;
  const int M = P.M;
  const int nkl = M * (M + 1) / 2;
  const int64_t gid = tk0;
  const int64_t pidx = P.act_post[P.act_post_off[M - 1] + gid / nkl];
  int l, k;
  kl_split((int)(gid % nkl), l, k);
  double* S = slice(P, th);
  const double* Wb = S + P.off_wbar + (int64_t)l * P.plane;
  const double* Wh = S + P.off_wobs + (int64_t)k * P.plane;
  Acc acc;
  acc_zero(acc);
  const int JM = P.Jl[M];
  int nsg = 0;
  for (int cc = 0; cc < JM; ++cc) {
    const int64_t leaf = pidx * JM + cc;
    nsg += (int)((P.leaf_poff[leaf + 1] - P.leaf_poff[leaf]) / T);
  }
  gemm_segs2(acc, nsg, [&](int sg) {
    int64_t leaf = pidx * JM;
    int nbl = (int)((P.leaf_poff[leaf + 1] - P.leaf_poff[leaf]) / T);
    while (sg >= nbl) {
      sg -= nbl;
      ++leaf;
      nbl = (int)((P.leaf_poff[leaf + 1] - P.leaf_poff[leaf]) / T);
    }
    const int64_t p = P.leaf_poff[leaf] + (int64_t)sg * T;
    return seg<Op::T, Op::N>(Wb + p * T, T, Wh + p * T, T, 1.0, round16(min(T, P.leaf_n[leaf] - T * sg)) / KC);
  }, lds);
  acc_store(acc, grad_of(P, S, M - 1, pidx).Tsum(l, k), T);
}

// ---------------------------------------------------------------- prior
// region (m, i), bottom-up: Cholesky adjoint of L_R, then the reverse row
// sweep of its knots
__global__ __launch_bounds__(NT, 2) void k_rprior(DevPlan P, const double* theta, int m, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_SWEEP];
  __shared__ double red[8];
  const int th = blockIdx.y;
  const int64_t i = P.act_post[P.act_post_off[m] + tk0];
  double* S = slice(P, th);
  const CovP c = load_cov(theta + 3 * th, P.cov);
  Grad gr = grad_of(P, S, m, i);
  double* reg = prior_reg(P, S, m, i);
  const double* L = reg + (int64_t)m * TT;
  const double* Li = reg + (int64_t)(m + 1) * TT;
  const double* X = knots_of(P, m, i);
  // The Cholesky adjoint keeps its intermediates in LDS (pitch PLD): each
  // product takes the previous result from there and streams its other
  // operand through the stage behind it.
  double* stage = lds + LDS_DOUBLES;
  // Lbar = -tril(Tsum^{m,m})
  const double* Tmm = gr.Tsum(m, m);
  {
    double v[TT / NT];   // all loads issued before the first store
#pragma unroll
    for (int j = 0; j < TT / NT; ++j) v[j] = Tmm[threadIdx.x + j * NT];
#pragma unroll
    for (int j = 0; j < TT / NT; ++j) {
      const int e = threadIdx.x + j * NT, r = e >> 6, q = e & 63;
      lds[r * PLD + q] = (q <= r) ? -v[j] : 0.0;
    }
  }
  __syncthreads();
  Acc acc;
  acc_zero(acc);
  gemm_lds_b(acc, L, T, true, lds, 1.0, stage);          // L' Lbar
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = acc_row(bi, v), q = acc_col(bj);
        if (q > r) acc.c[bi][bj][v] = 0.0;
        else if (q == r) acc.c[bi][bj][v] *= 0.5;       // Phi
      }
  acc_to_lds(acc, lds);
  __syncthreads();
  acc_zero(acc);
  gemm_lds_a(acc, lds, Li, T, true, 1.0, stage);        // Phi L^{-1}
  acc_to_lds(acc, lds);
  __syncthreads();
  acc_zero(acc);
  gemm_lds_b(acc, Li, T, true, lds, 1.0, stage);        // L^{-T} Phi L^{-1}
  acc_to_lds(acc, lds);
  __syncthreads();
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)                         // Wbar^m = sym(.)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = acc_row(bi, v), q = acc_col(bj);
        acc.c[bi][bj][v] = 0.5 * (lds[r * PLD + q] + lds[q * PLD + r]);
      }
  __syncthreads();
  acc_to_lds(acc, lds);
  __syncthreads();
  double g[3] = {0.0, 0.0, 0.0};
  acc_cov_contract(acc, X, P.rl[m], X, P.rl[m], c, false, g);
  // W^-bar^k = -Tsum^{m,k} - 2 Wbar^m W^^k_R, k < m
  for (int k = 0; k < m; ++k) {
    acc_load(acc, gr.Tsum(m, k), T);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc.c[bi][bj] = -acc.c[bi][bj];
    gemm_lds_a(acc, lds, reg + (int64_t)k * TT, T, true, -2.0, stage);
    acc_store(acc, gr.Wbar(k), T);
  }
  __syncthreads();
  row_sweep_reverse(P, S, c, X, P.rl[m], gr.Wbar(0), TT, m, i, g, lds, [&](Acc& acc, int l) { acc_load(acc, gr.Wbar(l), T); },
                    0, [&](int, int) { return Seg{}; });
  write_partial(P, S, P.n_sig_tiles + P.n_row_tasks + P.reg_base[m] + i, g, red);
}

// Tsum of a level-(m-1) region: sum over children (level m) of
// Tsum_c^{l,k} + Wbar_c^l' W^^k_c, k <= l <= m-1
__global__ __launch_bounds__(NT, 4) void k_rT(DevPlan P, int m, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int th = blockIdx.y;
  const int nkl = m * (m + 1) / 2;
  const int64_t gid = tk0;
  const int64_t pidx = P.act_post[P.act_post_off[m - 1] + gid / nkl];
  int l, k;
  kl_split((int)(gid % nkl), l, k);
  double* S = slice(P, th);
  const uint32_t cm = active_children(P, m, pidx);   // children with observations below them
  const int nch = __builtin_popcount(cm);
  Acc acc;
  acc_zero(acc);
  for (int cc = 0; cc < nch; ++cc) acc_load(acc, grad_of(P, S, m, nth_child(P, m, pidx, cm, cc)).Tsum(l, k), T, true);
  gemm_segs2(acc, nch, [&](int cc) {
    const int64_t ch = nth_child(P, m, pidx, cm, cc);
    return seg<Op::T, Op::N>(grad_of(P, S, m, ch).Wbar(l), T, prior_reg(P, S, m, ch) + (int64_t)k * TT, T, 1.0);
  }, lds);
  acc_store(acc, grad_of(P, S, m - 1, pidx).Tsum(l, k), T);
}

// sum of the partials in a fixed order: grad = (sum g0, sum g1, tau^2 sum g2)
__global__ __launch_bounds__(NT) void k_gsum(DevPlan P, const double* theta, double* out, int64_t nslot) {
  __shared__ double red[8];
  const int th = blockIdx.x;
  double* S = slice(P, th);
  double a = 0.0, b = 0.0, c = 0.0;
  // slots threadIdx.x, + NT, + 2 NT, ... in that order, eight loaded ahead
  for (int64_t q0 = threadIdx.x; q0 < nslot; q0 += 8 * NT) {
    double va[8], vb[8], vc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t q = q0 + (int64_t)u * NT;
      const double* o = S + P.off_gpart + (q < nslot ? q : 0) * 4;
      va[u] = o[0];
      vb[u] = o[1];
      vc[u] = o[2];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q0 + (int64_t)u * NT < nslot) {
        a += va[u];
        b += vb[u];
        c += vc[u];
      }
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    const double tau2 = exp(theta[3 * th + 2]);
    const bool bad = *(const unsigned long long*)(S + P.off_status) != 0ull;
    const double nan = __builtin_nan("");
    out[3 * th + 0] = bad ? nan : a;
    out[3 * th + 1] = bad ? nan : b;
    out[3 * th + 2] = bad ? nan : tau2 * c;
  }
}

__global__ void k_zero_gpart(DevPlan P, int64_t nslot) {
  double* S = slice(P, blockIdx.y);
  for (int64_t q = blockIdx.x * (int64_t)NT + threadIdx.x; q < nslot * 4; q += (int64_t)gridDim.x * NT)
    S[P.off_gpart + q] = 0.0;
}

// leaf solves of the reverse pass that only need the forward leaf factors:
// V = L_Sigma^{-T} Y and L_Sigma^{-1}; may run on a second stream while the
// posterior recursion proceeds
hipError_t launch_grad_leafsolve(const mra_plan_s& H, int nth, hipStream_t st, hipEvent_t after_v) {
  const DevPlan& P = H.dp;
  const PhaseFlops& F = H.pf;
  const int M = P.M;
  if (H.nchunks > 1) {   // MRA_CHECKPOINT: chunk by chunk in launch_grad_rest
    if (after_v) {
      const hipError_t e = hipEventRecord(after_v, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  Runner run{P, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  run.tuned(F_RLEAF_V, MAP_GROUPED, "rleaf_v", -1, F.rleaf_v, M + 1, nullptr, k_rleaf_v, 0,
            (int64_t)H.trsm_tasks.size() / 2);
  if (after_v) {
    const hipError_t e = hipEventRecord(after_v, st);
    if (e != hipSuccess) return e;
  }
  run.tuned(F_RLEAF_LINV, MAP_IDENTITY, "rleaf_linv", -1, F.rleaf_linv, 1, nullptr, k_rleaf_linv, 0,
            (int64_t)H.linv_tasks.size() / 2);
  return hipGetLastError();
}

// clear the gradient partial sums (any time before the reverse pass)
hipError_t launch_zero_gpart(const mra_plan_s& H, int nth, hipStream_t st) {
  const DevPlan& P = H.dp;
  const int M = P.M;
  const int64_t nrow = (int64_t)H.row_tasks.size() / 2;
  const int64_t nslot = P.n_sig_tiles + nrow + (M > 0 ? P.reg_base[M - 1] + P.nreg[M - 1] : 0);
  hipLaunchKernelGGL(k_zero_gpart, dim3(64, nth), dim3(NT), 0, st, P, nslot);
  return hipGetLastError();
}

// the posterior reverse pass (after the forward log-likelihood); clears the
// partial sums first unless the caller has done so
hipError_t launch_grad_post(const mra_plan_s& H, int nth, hipStream_t st, ForkHook* hook, bool zero_partials) {
  const DevPlan& P = H.dp;
  const PhaseFlops& F = H.pf;
  const int M = P.M;
  Runner run{P, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  hipError_t e;
  if (zero_partials && (e = launch_zero_gpart(H, nth, st)) != hipSuccess) return e;
  for (int m = 0; m < M; ++m) {
    run.tuned(F_RPOST, MAP_IDENTITY, "rpost", m, F.rpost[m], 1, nullptr, k_rpost, 0, H.nact_post(m), m);
    if (hook && (e = hook->at(M + 2 + m)) != hipSuccess) return e;
  }
  if (hook && (e = hook->at(0, true)) != hipSuccess) return e;
  return hipGetLastError();
}

// reverse leaf phase of leaf chunk c (MRA_CHECKPOINT), after its planes W^
// and Y have been recomputed: V = L^{-T} Y, L^{-1}, Q, Sigma-bar, W-bar and
// the level-(M-1) T-sums of the chunk
static void grad_leaf_chunk(const mra_plan_s& H, int c, const double* theta, int nth, double* grad_y, hipStream_t st) {
  const DevPlan P = chunk_plan(H, c);
  const PhaseFlops& F = H.pf;
  const int M = P.M;
  Runner run{P, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  const int64_t nrow = (int64_t)H.row_tasks.size() / 2, nsig = P.n_sig_tasks;
  const int64_t r0 = H.ck_row[c], r1 = H.ck_row[c + 1];
  const int64_t f0 = H.ck_fac[c], f1 = H.ck_fac[c + 1];
  const int64_t nlinv = (int64_t)H.linv_tasks.size() / 2, nfac = (int64_t)H.fac_tasks.size();
  auto sh = [](double f, int64_t a, int64_t b, int64_t n) { return n > 0 ? f * (double)(b - a) / (double)n : 0.0; };
  run.tuned(F_RLEAF_V, MAP_GROUPED, "rleaf_v", -1, sh(F.rleaf_v, f0, f1, nfac), M + 1, nullptr, k_rleaf_v,
            f0 * (M + 1), f1 * (M + 1));
  run.tuned(F_RLEAF_LINV, MAP_IDENTITY, "rleaf_linv", -1, sh(F.rleaf_linv, H.ck_linv[c], H.ck_linv[c + 1], nlinv), 1,
            nullptr, k_rleaf_linv, H.ck_linv[c], H.ck_linv[c + 1]);
  run.tuned(F_RLEAF_Q, MAP_CHUNKED, "rleaf_q", -1, sh(F.rleaf_q, r0, r1, nrow), M + 1, nullptr, k_rleaf_q,
            r0 * (M + 1), r1 * (M + 1), grad_y);
  run.tuned(F_RLEAF_SBAR, MAP_IDENTITY, "rleaf_sbar", -1, sh(F.rleaf_sbar, H.ck_sig[c], H.ck_sig[c + 1], nsig), 1,
            nullptr, k_rleaf_sbar, H.ck_sig[c], H.ck_sig[c + 1], theta);
  run.tuned(F_RROWS, MAP_CHUNKED, "rrows_leaf", -1, sh(F.rrows + F.rleaf_wbar, r0, r1, nrow), 1, nullptr,
            k_rrows_leaf, r0, r1, theta);
  const int nkl = M * (M + 1) / 2;
  const int64_t nq = H.nact_post(M - 1);
  run.tuned(F_RT_LEAF, MAP_GROUPED, "rT_leaf", -1, sh(F.rT_leaf, H.ck_actq[c], H.ck_actq[c + 1], nq), nkl, nullptr,
            k_rT_leaf, H.ck_actq[c] * nkl, H.ck_actq[c + 1] * nkl);
}

// the leaf and prior reverse passes and the final sum (after both of the above)
hipError_t launch_grad_rest(const mra_plan_s& H, const double* y, int64_t y_stride, const double* theta, int nth,
                            double* out_grad, double* grad_y, hipStream_t st, hipEvent_t wait_linv) {
  const DevPlan& P = H.dp;
  const PhaseFlops& F = H.pf;
  const int M = P.M;
  Runner run{P, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  const int64_t nrow = (int64_t)H.row_tasks.size() / 2;
  const int64_t nslot = P.n_sig_tiles + nrow + (M > 0 ? P.reg_base[M - 1] + P.nreg[M - 1] : 0);
  if (H.nchunks > 1) {
    // MRA_CHECKPOINT: recompute each chunk's W^ and Y from the stored prior
    // blocks and leaf factors, then run its reverse leaf phase
    for (int c = 0; c < H.nchunks; ++c) {
      const hipError_t e = launch_leaf_planes(H, c, y, theta, nth, st, y_stride, false);
      if (e != hipSuccess) return e;
      grad_leaf_chunk(H, c, theta, nth, grad_y, st);
    }
  } else {
    run.tuned(F_RLEAF_Q, MAP_CHUNKED, "rleaf_q", -1, F.rleaf_q, M + 1, nullptr, k_rleaf_q, 0, nrow * (M + 1),
              grad_y);
    if (wait_linv) {
      const hipError_t e = hipStreamWaitEvent(st, wait_linv, 0);
      if (e != hipSuccess) return e;
    }
    run.tuned(F_RLEAF_SBAR, MAP_IDENTITY, "rleaf_sbar", -1, F.rleaf_sbar, 1, nullptr, k_rleaf_sbar, 0, P.n_sig_tasks,
              theta);
    if (M > 0) {
      run.tuned(F_RROWS, MAP_CHUNKED, "rrows_leaf", -1, F.rrows + F.rleaf_wbar, 1, H.cut_rrows, k_rrows_leaf, 0, nrow,
                theta);
      const int nkl = M * (M + 1) / 2;
      run.tuned(F_RT_LEAF, MAP_GROUPED, "rT_leaf", -1, F.rT_leaf, nkl, nullptr, k_rT_leaf, 0,
                H.nact_post(M - 1) * (int64_t)nkl);
    }
  }
  if (M > 0) {
    for (int m = M - 1; m >= 0; --m) {
      run.tuned(F_RPRIOR, MAP_IDENTITY, "rprior", m, F.rprior[m], 1, nullptr, k_rprior, 0, H.nact_post(m), theta, m);
      if (m > 0)
        run.tuned(F_RT, MAP_GROUPED, "rT", m, F.rT[m], m * (m + 1) / 2, nullptr, k_rT, 0,
                  H.nact_post(m - 1) * (int64_t)(m * (m + 1) / 2), m);
    }
  }
  hipLaunchKernelGGL(k_gsum, dim3(nth), dim3(NT), 0, st, P, theta, out_grad, nslot);
  return hipGetLastError();
}

}  // namespace mra
