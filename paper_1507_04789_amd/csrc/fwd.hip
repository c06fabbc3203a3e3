// Forward M-RA kernels: prior quantities (eq. priorw), leaf quantities
// (eq. helpquantities at m = M), posterior recursion (eq. posterior,
// mainquantities, helpquantities) and the log-likelihood (Sec. 3.3).
//
// Whitened form.  With K_a^{-1} = W^{level(a)}_a = L_a L_a', the blocks
// W^^k_R = W^k_R L_{a_k}^{-T} turn eq. priorw into a block Cholesky along
// each chain of regions:
//   W^l_R = C_0(Q_R, Q_{a_l}) - sum_{k<l} W^^k_R W^^k_{a_l}',
//   W^^l_R = W^l_R L_{a_l}^{-T},   L_R = chol(W^m_R).
// The weights xi_a = L_a' eta_a are then N(0, I), the leaf basis rows are
// W^^k_R, and the posterior precision of xi_R given the finer levels is
// I + A^{m,m}_R (the whitened K~^{-1}).  log|K~^{-1}| - log|K^{-1}| =
// log|I + A^{m,m}|, so the d and u recursions of Sec. 3.3 keep their form.
#include "common.hpp"
#include "plan.hpp"
#include "launch.hpp"

namespace mra {

// ------------------------------------------------------------------ kernels

// zero the per-theta status word and leaf log-determinants
__global__ void k_init(DevPlan P) {
  double* S = slice(P, blockIdx.y);
  for (int64_t q = blockIdx.x * (int64_t)NT + threadIdx.x; q < P.n_leaves; q += (int64_t)gridDim.x * NT)
    S[P.off_leafd + q] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x < 4) S[P.off_status + threadIdx.x] = 0.0;
}

// plane M of the leaf rows [p_begin, p_end): z in column 0 (leaf order,
// padded), the trend columns X[j] (caller's order, [px][n]) in columns
// 1..px, zero elsewhere; parameter row b reads its data at y + b * y_stride
__global__ void k_gather(DevPlan P, const double* y, int64_t y_stride, int64_t p_begin, int64_t p_end,
                         const double* X, int px) {
  double* S = slice(P, blockIdx.y);
  y += blockIdx.y * y_stride;
  double* zp = S + P.off_wobs + (int64_t)P.M * P.plane + p_begin * T;
  const int64_t ne = (p_end - p_begin) * T;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < ne; e += (int64_t)gridDim.x * NT) {
    int64_t p = p_begin + (e >> 6);
    int col = (int)(e & 63);
    int64_t g = P.obs_gidx[p];
    double v = 0.0;
    if (g >= 0) {
      if (col == 0) v = y[g];
      else if (col <= px) v = X[(int64_t)(col - 1) * P.n + g];
    }
    zp[e] = v;
  }
}

// prior level m < M: one workgroup per region
__global__ __launch_bounds__(NT, 2) void k_prior(DevPlan P, const double* theta, int m, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  __shared__ double lds_x[T * PLD];
  const int th = blockIdx.y;
  const int64_t i = P.act_prior[P.act_prior_off[m] + tk0];
  double* S = slice(P, th);
  const CovP c = load_cov(theta + 3 * th, P.cov);
  double* reg = prior_reg(P, S, m, i);
  const double* X = knots_of(P, m, i);
  const int rm = P.rl[m];
  row_sweep(P, S, c, X, rm, reg, TT, m, i, lds, lds_x);   // lds_x is free until the factorisation
  Acc acc;
  acc_cov(acc, X, rm, X, rm, c, true, 0.0);
  gemm_segs2(acc, m, [&](int k) { return seg<Op::N, Op::T>(reg + k * TT, T, reg + k * TT, T, -1.0); }, lds,
            round16(rm));
  acc_to_lds(acc, lds);
  __syncthreads();
  if (!potrf_trtri(lds, lds_x, reg + (m + 1) * TT) && threadIdx.x == 0) record_failure(P, S, m, i);
  lds_to_global(lds, reg + m * TT);
}

// rows of W^ for the observations of one 64-row leaf tile
__global__ __launch_bounds__(NT, 2) void k_leaf_rows(DevPlan P, const double* theta, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_SWEEP];
  const int th = blockIdx.y;
  const int32_t* task = P.row_tasks + 2 * tk0;
  const int leaf = task[0];
  const int64_t p0 = task[1];
  double* S = slice(P, th);
  const CovP c = load_cov(theta + 3 * th, P.cov);
  const int nx = min(T, (int)(P.leaf_n[leaf] - (p0 - P.leaf_poff[leaf])));
  row_sweep(P, S, c, P.obs_xy + 2 * p0, nx, S + P.off_wobs + p0 * T, P.plane, P.M, leaf, lds, lds + LDS_DOUBLES);
}

// Sigma_R = C_0(S_R, S_R) + tau^2 I - W^_R W^_R' per tile (bi >= bj)
__global__ __launch_bounds__(NT) void k_sigma(DevPlan P, const double* theta, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int th = blockIdx.y;
  const int32_t* task = P.sig_tasks + 3 * tk0;
  const int leaf = task[0], bi = task[1], bj = task[2];
  double* S = slice(P, th);
  const CovP c = load_cov(theta + 3 * th, P.cov);
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  const int nR = P.leaf_n[leaf];
  const int64_t pi = poff + (int64_t)T * bi, pj = poff + (int64_t)T * bj;
  const int nvi = min(T, nR - T * bi), nvj = min(T, nR - T * bj);
  Acc acc;
  acc_cov(acc, P.obs_xy + 2 * pi, nvi, P.obs_xy + 2 * pj, nvj, c, bi == bj, c.tau2);
  const double* W = S + P.off_wobs;
  gemm_segs2(acc, P.M,
            [&](int k) { return seg<Op::N, Op::T>(W + k * P.plane + pi * T, T, W + k * P.plane + pj * T, T, -1.0); },
            lds, round16(nvi), round16(nvj));
  acc_store(acc, S + P.off_sig + (P.leaf_soff[leaf] + (int64_t)bi * nb + bj) * TT, T);
}

// blocked left-looking Cholesky of one leaf's Sigma (tiles in place), the
// inverses of its diagonal tiles, and d_R = log|Sigma_R|
__global__ __launch_bounds__(NT, 2) void k_leaf_potrf(DevPlan P, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  __shared__ double lds_x[T * PLD];
  __shared__ double red[8];
  const int th = blockIdx.y;
  const int leaf = P.fac_tasks[tk0];
  double* S = slice(P, th);
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  bool ok = true;
  const double logdet = potrf_tiles(S + P.off_sig + P.leaf_soff[leaf] * TT, S + P.off_dinv + P.leaf_doff[leaf] * TT, nb,
                                    P.leaf_n[leaf], lds, lds_x, red, ok);
  if (threadIdx.x == 0) {
    S[P.off_leafd + leaf] = logdet;
    if (!ok) record_failure(P, S, P.M, leaf);
  }
}

// Y = L_Sigma^{-1} X for one column plane of one leaf (forward substitution
// by tiles with the inverted diagonal tiles).  The data plane M holds zc
// nonzero columns (a multiple of 16: z and the trend columns); the others
// stay zero and are not multiplied.  RES (the launch for the large leaves):
// after the updates, the right-hand side tile stays in LDS for the product
// with the diagonal inverse instead of a round trip through global memory
// (same products in the same order, so the same bits; more LDS per block).
template <bool RES>
__global__ __launch_bounds__(NT, 4) void k_leaf_trsm(DevPlan P, int zc, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[RES ? LDS_SWEEP : LDS_DOUBLES];
  const int th = blockIdx.y;
  const int32_t* task = P.trsm_tasks + 2 * tk0;
  const int leaf = task[0], cpl = task[1];
  double* S = slice(P, th);
  const int64_t poff = P.leaf_poff[leaf];
  const int nb = (int)((P.leaf_poff[leaf + 1] - poff) / T);
  const double* base = S + P.off_sig + P.leaf_soff[leaf] * TT;
  const double* dinv = S + P.off_dinv + P.leaf_doff[leaf] * TT;
  const double* X = S + P.off_wobs + cpl * P.plane + poff * T;
  double* Y = S + P.off_y + cpl * P.plane + poff * T;
  const int nR = P.leaf_n[leaf];
  const int nc = cpl == P.M ? zc : T;
  Acc acc;
  for (int ib = 0; ib < nb; ++ib) {
    const int mr = round16(min(T, nR - T * ib));
    const double* R = X + (int64_t)ib * TT;   // right-hand side after the updates
    if (ib > 0) {
      acc_load(acc, R, T);
      gemm_segs2(acc, ib,
                [&](int jb) { return seg<Op::N, Op::N>(base + ((int64_t)ib * nb + jb) * TT, T, Y + (int64_t)jb * TT, T, -1.0); },
                lds, mr, nc);
      if (RES) {
        acc_to_lds(acc, lds);
        __syncthreads();
        acc_zero(acc);
        gemm_lds_b(acc, dinv + (int64_t)ib * TT, T, false, lds, 1.0, lds + LDS_DOUBLES, mr, nc);
        acc_store(acc, Y + (int64_t)ib * TT, T);
        __syncthreads();
        continue;
      }
      acc_store(acc, Y + (int64_t)ib * TT, T);
      __syncthreads();
      R = Y + (int64_t)ib * TT;
    }
    acc_zero(acc);
    gemm_segs(acc, 1, [&](int) { return seg<Op::N, Op::N>(dinv + (int64_t)ib * TT, T, R, T, 1.0); }, lds, mr, nc);
    acc_store(acc, Y + (int64_t)ib * TT, T);
    __syncthreads();
  }
}

// leaf products summed over the J leaves of a level-(M-1) region
// (eq. helpquantities at m = M, eq. mainquantities):
//   A^{k,l} = sum_c Y^k_c' Y^l_c, w^k = sum_c Y^k_c' y_c, u = sum_c y_c'y_c, d = sum_c d_c
__global__ __launch_bounds__(NT) void k_leaf_reduce(DevPlan P, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  __shared__ double red[8];
  const int th = blockIdx.y;
  const int M = P.M;
  const int nkl = M * (M + 1) / 2;
  const int64_t gid = tk0;
  const int64_t pidx = P.reduce_order[gid / nkl];
  const int kl = (int)(gid % nkl);
  int k, l;
  kl_split(kl, k, l);
  double* S = slice(P, th);
  Post po = post_of(P, S, M - 1, pidx);
  const double* Yk = S + P.off_y + k * P.plane;
  const double* Yl = S + P.off_y + l * P.plane;
  const double* Yz = S + P.off_y + (int64_t)M * P.plane;
  Acc acc;
  acc_zero(acc);
  // segments: the row blocks of the J_M children, K = valid rows rounded to 16
  const int JM = P.Jl[M];
  int nsg = 0;
  for (int c = 0; c < JM; ++c) {
    const int64_t leaf = pidx * JM + c;
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
    const int rows = min(T, P.leaf_n[leaf] - T * sg);
    return seg<Op::T, Op::N>(Yk + p * T, T, Yl + p * T, T, 1.0, round16(rows) / KC);
  }, lds);
  acc_store(acc, po.A(k, l), T);
  if (k == l) {      // w^k = sum_c Y^k_c' y_c: column threadIdx & 63, rows split over the waves
    const int col = threadIdx.x & 63;
    double w[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < JM; ++c) {
      const int64_t leaf = pidx * JM + c;
      const int64_t end = P.leaf_poff[leaf] + P.leaf_n[leaf];
      int64_t p = P.leaf_poff[leaf] + wave_id();
      for (; p + 12 < end; p += 16) {   // four rows in flight
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] += Yk[(p + 4 * q) * T + col] * Yz[(p + 4 * q) * T];
      }
      for (; p < end; p += 4) w[0] += Yk[p * T + col] * Yz[p * T];
    }
    const double ws = wave_col_sum((w[0] + w[1]) + (w[2] + w[3]), lds);
    if (threadIdx.x < T) po.omega(k)[threadIdx.x] = ws;
  }
  if (kl == 0) {
    double u = 0.0;
    for (int c = 0; c < JM; ++c) {
      const int64_t leaf = pidx * JM + c;
      for (int64_t p = P.leaf_poff[leaf] + threadIdx.x; p < P.leaf_poff[leaf] + P.leaf_n[leaf]; p += NT)
        u += Yz[p * T] * Yz[p * T];
    }
    u = block_sum(u, red);
    if (threadIdx.x == 0) {
      double dsum = 0.0;
      for (int c = 0; c < JM; ++c) dsum += S[P.off_leafd + pidx * JM + c];
      *po.d() = dsum;
      *po.u() = u;
    }
  }
}

// posterior level m: K~^{-1} = I + A^{m,m} (whitened), its factor and
// inverse, Z = Lt^{-1} [A^{m,0..m-1} | w^m], d and u (Sec. 3.3)
__global__ __launch_bounds__(NT, 2) void k_post(DevPlan P, int m, double* out_loglik, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  __shared__ double lds_x[T * PLD];
  __shared__ double red[8];
  __shared__ double wsh[T];
  const int th = blockIdx.y;
  const int64_t i = P.act_post[P.act_post_off[m] + tk0];
  double* S = slice(P, th);
  Post po = post_of(P, S, m, i);
  if (threadIdx.x < T) wsh[threadIdx.x] = po.omega(m)[threadIdx.x];
  tile_to_lds(po.A(m, m), T, lds);
  __syncthreads();
  if (threadIdx.x < T) lds[threadIdx.x * PLD + threadIdx.x] += 1.0;
  __syncthreads();
  const bool ok = potrf_trtri(lds, lds_x, po.Lti());
  const double ld = 2.0 * logdiag_lds(lds, T, red);
  // Z_l = Lt^{-1} A^{m,l}: the inverse is still in lds_x (pitch PLD)
  Acc acc;
  for (int l = 0; l < m; ++l) {
    acc_zero(acc);
    gemm_lds_a(acc, lds_x, po.A(m, l), T, true, 1.0, lds);
    acc_store(acc, po.Z(l), T);
  }
  double zq = 0.0;
  if (threadIdx.x < T) {
    const double* Li = lds_x + threadIdx.x * PLD;
    for (int q = 0; q <= (int)threadIdx.x; ++q) zq += Li[q] * wsh[q];
    po.zw()[threadIdx.x] = zq;
  }
  const double nrm = block_sum(zq * zq, red);
  if (threadIdx.x == 0) {
    const double dR = *po.d() + ld;
    const double uR = *po.u() - nrm;
    *po.d() = dR;
    *po.u() = uR;
    if (!ok) record_failure(P, S, m, i);
    if (m == 0) {
      const double ll = -0.5 * (dR + uR) - 0.5 * (double)P.n * 1.8378770664093453;
      S[P.off_scal] = ll;
      if (out_loglik) out_loglik[th] = ll;
    }
  }
}

// child sums for level m-1 (eq. mainquantities with eq. helpquantities):
//   A^{k,l}_P = sum_c (A^{k,l}_c - Z^k_c' Z^l_c),  w^k_P = sum_c (w^k_c - Z^k_c' z_c)
__global__ __launch_bounds__(NT, 4) void k_post_reduce(DevPlan P, int m, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int th = blockIdx.y;
  const int nkl = m * (m + 1) / 2;       // blocks k >= l <= m-1
  const int64_t gid = tk0;
  const int64_t pidx = P.act_post[P.act_post_off[m - 1] + gid / nkl];
  const int kl = (int)(gid % nkl);
  int k, l;
  kl_split(kl, k, l);
  double* S = slice(P, th);
  Post pp = post_of(P, S, m - 1, pidx);
  // children with observations below them (the others contribute zero)
  const uint32_t cm = active_children(P, m, pidx);
  const int nch = __builtin_popcount(cm);
  Acc acc;
  acc_zero(acc);
  for (int c = 0; c < nch; ++c) acc_load(acc, post_of(P, S, m, nth_child(P, m, pidx, cm, c)).A(k, l), T, true);
  gemm_segs2(acc, nch, [&](int c) {
    Post pc = post_of(P, S, m, nth_child(P, m, pidx, cm, c));
    return seg<Op::T, Op::N>(pc.Z(k), T, pc.Z(l), T, -1.0);
  }, lds);
  acc_store(acc, pp.A(k, l), T);
  if (k == l) {      // w^k_P = sum_c (w^k_c - Z^k_c' z_c)
    double w = 0.0;
    const int col = threadIdx.x & 63;
    for (int c = 0; c < nch; ++c) {
      Post pc = post_of(P, S, m, nth_child(P, m, pidx, cm, c));
      const double* Zk = pc.Z(k);
      const double* zw = pc.zw();
      double zk[T / 4], zv[T / 4];   // rows wave, wave + 4, ...: all loads issued first
#pragma unroll
      for (int j = 0; j < T / 4; ++j) {
        zk[j] = Zk[(wave_id() + 4 * j) * T + col];
        zv[j] = zw[wave_id() + 4 * j];
      }
      if (wave_id() == 0) w += pc.omega(k)[col];
#pragma unroll
      for (int j = 0; j < T / 4; ++j) w -= zk[j] * zv[j];
    }
    w = wave_col_sum(w, lds);
    if (threadIdx.x < T) pp.omega(k)[threadIdx.x] = w;
  }
  if (kl == 0 && wave_id() == 0) {   // lane c loads child c's d and u; summed in child order
    const int c = lane_id();
    double dv = 0.0, uv = 0.0;
    if (c < nch) {
      Post pc = post_of(P, S, m, nth_child(P, m, pidx, cm, c));
      dv = *pc.d();
      uv = *pc.u();
    }
    double dsum = 0.0, usum = 0.0;
    for (int q = 0; q < nch; ++q) {
      dsum += readlane_d(dv, q);
      usum += readlane_d(uv, q);
    }
    if (c == 0) {
      *pp.d() = dsum;
      *pp.u() = usum;
    }
  }
}

// M = 0: the single leaf is the root (exact Gaussian likelihood)
__global__ __launch_bounds__(NT) void k_root_leaf(DevPlan P, double* out_loglik) {
  __shared__ double red[8];
  const int th = blockIdx.y;
  double* S = slice(P, th);
  const double* Yz = S + P.off_y;   // plane 0 = plane M
  double u = 0.0;
  for (int64_t p = threadIdx.x; p < P.npad; p += NT) u += Yz[p * T] * Yz[p * T];
  u = block_sum(u, red);
  if (threadIdx.x == 0) {
    const double dR = S[P.off_leafd];
    const double ll = -0.5 * (dR + u) - 0.5 * (double)P.n * 1.8378770664093453;
    S[P.off_scal] = ll;
    if (out_loglik) out_loglik[th] = ll;
  }
}

// NaN for parameter vectors whose factorisations broke down
__global__ void k_mark_failed(DevPlan P, double* out, int width) {
  const int th = blockIdx.x;
  const double* S = slice(P, th);
  if (*(const unsigned long long*)(S + P.off_status) != 0ull && threadIdx.x < width)
    out[th * width + threadIdx.x] = __builtin_nan("");
}

// ------------------------------------------------------------------ launches

// Device plan for leaf chunk c (MRA_CHECKPOINT): the plane buffers hold only
// the chunk's rows and the L^{-1} buffer only its leaves' tiles, so their
// offsets are shifted back by the chunk's first row and first tile; every
// kernel then addresses them with global row and tile indices.  The whole
// plan when there is a single chunk.
DevPlan chunk_plan(const mra_plan_s& H, int c) {
  DevPlan P = H.dp;
  if (H.nchunks > 1) {
    const int64_t sh = H.chunk_row[c] * T;
    P.off_wobs -= sh;
    P.off_y -= sh;
    P.off_v -= sh;
    P.off_q -= sh;
    P.off_wbar -= sh;
    P.off_linv -= H.ck_soff[c] * TT;
  }
  return P;
}

// nonzero columns of the data plane, rounded up to the 16-column MFMA block:
// z and px trend columns
static int zcols(int px) { return (px + 1 + 15) / 16 * 16; }

// share of a whole-plan flop count carried by the tasks [a, b) of n
static double share(double f, int64_t a, int64_t b, int64_t n) { return n > 0 ? f * (double)(b - a) / (double)n : 0.0; }

// data plane of chunk c (z in column 0 of plane M)
static void gather_chunk(const mra_plan_s& H, const DevPlan& P, int c, const double* y, int64_t y_stride, int nth,
                         hipStream_t st, const double* X, int px) {
  const int64_t p0 = H.chunk_row[c], p1 = H.chunk_row[c + 1];
  if (p1 <= p0) return;
  int64_t gx = ((p1 - p0) * T + NT - 1) / NT;
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)gx, nth), dim3(NT), 0, st, P, y, y_stride, p0, p1, X, px);
}

// The leaf planes of chunk c: the data plane, the basis rows W^ (eq. priorw
// at level M) and Y = L_Sigma^{-1} [W^ | z].  With factor = true also the
// leaf covariances and their factors (forward pass); otherwise the stored
// factors are used and the work is recomputation (flops not counted).
hipError_t launch_leaf_planes(const mra_plan_s& H, int c, const double* y, const double* theta, int nth,
                              hipStream_t st, int64_t y_stride, bool factor, const double* X, int px) {
  const DevPlan P = chunk_plan(H, c);
  const PhaseFlops& F = H.pf;
  const int M = P.M;
  Runner run{P, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  const int64_t nrow = (int64_t)H.row_tasks.size() / 2, nsig = (int64_t)H.sig_tasks.size() / 3;
  gather_chunk(H, P, c, y, y_stride, nth, st, X, px);
  const int64_t r0 = H.ck_row[c], r1 = H.ck_row[c + 1];
  run.tuned(F_LEAF_ROWS, MAP_CHUNKED, factor ? "leaf_rows" : "leaf_rows_re", -1,
            factor ? share(F.leaf_rows, r0, r1, nrow) : 0.0, 1, nullptr, k_leaf_rows, r0, r1, theta);
  const int64_t f0 = H.ck_fac[c], f1 = H.ck_fac[c + 1];
  if (factor) {
    run.tuned(F_SIGMA, MAP_IDENTITY, "leaf_sigma", -1, share(F.sigma, H.ck_sig[c], H.ck_sig[c + 1], nsig), 1, nullptr,
              k_sigma, H.ck_sig[c], H.ck_sig[c + 1], theta);
    run.tuned(F_POTRF, MAP_IDENTITY, "leaf_potrf", -1, H.potrf_flops_big(f1) - H.potrf_flops_big(f0), 1, nullptr,
              k_leaf_potrf, f0, f1);
  }
  run.tuned(F_TRSM, MAP_GROUPED, factor ? "leaf_trsm" : "leaf_trsm_re", -1,
            factor ? H.trsm_flops_big(f1) - H.trsm_flops_big(f0) : 0.0, M + 1, nullptr, k_leaf_trsm<false>, f0 * (M + 1),
            f1 * (M + 1), zcols(px));
  return hipGetLastError();
}

// init, prior levels and the leaf factorisation (everything the reverse
// pass's leaf solves depend on).  With a side stream, the leaves of
// big_tiles tiles or more are factored and solved there while the small
// leaves proceed on `st`; side->big marks their completion and is awaited in
// launch_forward_back.  With MRA_CHECKPOINT the leaf phase and the leaf
// products run chunk by chunk here (no side stream).
// plane M of every leaf row: the data (and trend columns) in leaf order
static void launch_gather(const mra_plan_s& H, const double* y, int64_t y_stride, int nth, hipStream_t st,
                          const double* X, int px) {
  const DevPlan& P = H.dp;
  int64_t gx = (P.npad * T + NT - 1) / NT;
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)gx, nth), dim3(NT), 0, st, P, y, y_stride, (int64_t)0, P.npad, X, px);
}

hipError_t launch_forward_front(const mra_plan_s& H, const double* y, const double* theta, int nth, hipStream_t st,
                                const Side* side, int64_t y_stride, const double* X, int px) {
  const DevPlan& P = H.dp;
  const PhaseFlops& F = H.pf;
  const int M = P.M;
  Runner run{P, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  // the data plane is first read by the leaf solves: with a second stream its
  // gather runs there, beside the prior recursion's narrow top levels
  const bool side_gather = side && H.nchunks == 1;
  if (side_gather) {
    hipError_t e;
    if ((e = hipEventRecord(side->gfork, st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(side->s, side->gfork, 0)) != hipSuccess) return e;
    launch_gather(H, y, y_stride, nth, side->s, X, px);
    if ((e = hipEventRecord(side->gath, side->s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_init, dim3(64, nth), dim3(NT), 0, st, P);
  for (int m = 0; m < M; ++m)
    run.tuned(F_PRIOR, MAP_IDENTITY, "prior", m, F.prior[m], 1, nullptr, k_prior, 0, H.nact_prior(m), theta, m);
  if (H.nchunks > 1) {
    const int nkl = M * (M + 1) / 2;
    const int64_t nred = (int64_t)H.reduce_order.size();
    for (int c = 0; c < H.nchunks; ++c) {
      hipError_t e = launch_leaf_planes(H, c, y, theta, nth, st, y_stride, true, X, px);
      if (e != hipSuccess) return e;
      const DevPlan Pc = chunk_plan(H, c);
      Runner rc{Pc, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
      rc.tuned(F_LEAF_REDUCE, MAP_GROUPED, "leaf_reduce", -1, share(F.leaf_reduce, H.ck_red[c], H.ck_red[c + 1], nred),
               nkl, nullptr, k_leaf_reduce, H.ck_red[c] * nkl, H.ck_red[c + 1] * nkl);
      if (X && (e = launch_gls_leaf(H, Pc, H.ck_red[c], H.ck_red[c + 1], px + 1, st)) != hipSuccess) return e;
    }
    return hipGetLastError();
  }
  if (!side_gather) launch_gather(H, y, y_stride, nth, st, X, px);
  run.tuned(F_LEAF_ROWS, MAP_CHUNKED, "leaf_rows", -1, F.leaf_rows, 1, nullptr, k_leaf_rows, 0,
            (int64_t)H.row_tasks.size() / 2, theta);
  run.tuned(F_SIGMA, MAP_IDENTITY, "leaf_sigma", -1, F.sigma, 1, nullptr, k_sigma, 0, (int64_t)H.sig_tasks.size() / 3,
            theta);
  const int64_t nfac = (int64_t)H.fac_tasks.size(), ntrsm = (int64_t)H.trsm_tasks.size() / 2;
  const int64_t nbig = side ? H.nbig() : 0;
  if (nbig > 0) {
    hipError_t e;
    if ((e = hipEventRecord(side->fork, st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(side->s, side->fork, 0)) != hipSuccess) return e;
    Runner rs{P, nth, side->s, false, H.prof, H.tune};
    const double fpb = H.potrf_flops_big(nbig), ftb = H.trsm_flops_big(nbig);
    rs.tuned(F_POTRF, MAP_IDENTITY, "leaf_potrf_big", -1, fpb, 1, nullptr, k_leaf_potrf, 0, nbig);
    rs.tuned(F_TRSM, MAP_GROUPED, "leaf_trsm_big", -1, ftb, M + 1, nullptr, k_leaf_trsm<true>, 0, nbig * (M + 1),
             zcols(px));
    if ((e = hipEventRecord(side->big, side->s)) != hipSuccess) return e;
  }
  run.tuned(F_POTRF, MAP_IDENTITY, "leaf_potrf", -1, F.potrf - H.potrf_flops_big(nbig), 1, nullptr, k_leaf_potrf, nbig,
            nfac);
  if (side_gather) {
    const hipError_t e = hipStreamWaitEvent(st, side->gath, 0);
    if (e != hipSuccess) return e;
  }
  run.tuned(F_TRSM, MAP_GROUPED, "leaf_trsm", -1, F.trsm - H.trsm_flops_big(nbig), M + 1, nullptr, k_leaf_trsm<false>,
            nbig * (M + 1), ntrsm, zcols(px));
  return hipGetLastError();
}

// leaf products, posterior recursion and the log-likelihood.  With large
// leaves on the side stream, the parents whose children are all small go
// first; the main stream then waits for the large leaves.
hipError_t launch_forward_back(const mra_plan_s& H, int nth, double* out_loglik, hipStream_t st, const Side* side,
                               ForkHook* hook) {
  const DevPlan& P = H.dp;
  const PhaseFlops& F = H.pf;
  const int M = P.M;
  Runner run{P, nth, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  const bool split = side && H.nbig() > 0;
  auto at = [&](int stage) -> hipError_t { return hook ? hook->at(stage) : hipSuccess; };
  hipError_t e = at(0);
  if (e != hipSuccess) return e;
  if (H.nchunks > 1) {   // leaf products already formed chunk by chunk
    if ((e = at(1)) != hipSuccess) return e;
    for (int m = M - 1; m >= 0; --m) {
      run.tuned(F_POST, MAP_IDENTITY, "post", m, F.post[m], 1, nullptr, k_post, 0, H.nact_post(m), m, out_loglik);
      if (m > 0)
        run.tuned(F_POST_REDUCE, MAP_GROUPED, "post_reduce", m, F.post_reduce[m], m * (m + 1) / 2, nullptr,
                  k_post_reduce, 0, H.nact_post(m - 1) * (int64_t)(m * (m + 1) / 2), m);
      if ((e = at(1 + M - m)) != hipSuccess) return e;
    }
  } else if (M == 0) {
    if (split && (e = hipStreamWaitEvent(st, side->big, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_root_leaf, dim3(1, nth), dim3(NT), 0, st, P, out_loglik);
  } else {
    const int nkl = M * (M + 1) / 2;
    const int64_t ntask = (int64_t)H.reduce_order.size() * nkl;
    const int64_t cut = split ? H.nsmall() * nkl : ntask;
    const double f0 = ntask ? F.leaf_reduce * (double)cut / (double)ntask : 0.0;
    run.tuned(F_LEAF_REDUCE, MAP_GROUPED, "leaf_reduce", -1, f0, nkl, nullptr, k_leaf_reduce, 0, cut);
    if (split) {
      if ((e = hipStreamWaitEvent(st, side->big, 0)) != hipSuccess) return e;
      run.tuned(F_LEAF_REDUCE, MAP_GROUPED, "leaf_reduce_big", -1, F.leaf_reduce - f0, nkl, nullptr, k_leaf_reduce,
                cut, ntask);
    }
    if ((e = at(1)) != hipSuccess) return e;
    for (int m = M - 1; m >= 0; --m) {
      run.tuned(F_POST, MAP_IDENTITY, "post", m, F.post[m], 1, nullptr, k_post, 0, H.nact_post(m), m, out_loglik);
      if (m > 0)
        run.tuned(F_POST_REDUCE, MAP_GROUPED, "post_reduce", m, F.post_reduce[m], m * (m + 1) / 2, nullptr,
                  k_post_reduce, 0, H.nact_post(m - 1) * (int64_t)(m * (m + 1) / 2), m);
      if ((e = at(1 + M - m)) != hipSuccess) return e;
    }
  }
  if (out_loglik) hipLaunchKernelGGL(k_mark_failed, dim3(nth), dim3(64), 0, st, P, out_loglik, 1);
  if (M == 0 && (e = at(M + 1)) != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_forward(const mra_plan_s& H, const double* y, const double* theta, int nth, double* out_loglik,
                          hipStream_t st) {
  hipError_t e = launch_forward_front(H, y, theta, nth, st);
  if (e != hipSuccess) return e;
  return launch_forward_back(H, nth, out_loglik, st);
}

}  // namespace mra
