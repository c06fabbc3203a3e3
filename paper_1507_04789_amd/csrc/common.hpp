// Device helpers shared by the forward, reverse and prediction kernels:
// arena addressing of the per-region storage and the row sweep of eq. priorw.
#pragma once
#include "cov.hpp"

namespace mra {

__device__ __forceinline__ double* slice(const DevPlan& P, int th) { return P.work + (int64_t)th * P.theta_stride; }

// Region storage is compact over the active regions of a level (regions
// with nothing below them are pruned); callers only pass active regions.
__device__ __forceinline__ double* prior_reg(const DevPlan& P, double* S, int m, int64_t i) {
  return S + P.prior_off[m] + (int64_t)P.slot_prior[P.reg_base[m] + i] * (m + 2) * TT;
}
__device__ __forceinline__ bool post_active(const DevPlan& P, int m, int64_t i) {
  return P.slot_post[P.reg_base[m] + i] >= 0;
}
__device__ __forceinline__ const double* knots_of(const DevPlan& P, int m, int64_t i) {
  return P.knot_xy + (P.reg_base[m] + i) * (2 * T);
}
__device__ __forceinline__ int64_t ancestor(const DevPlan& P, int m, int64_t i, int l) {
  for (int q = m; q > l; --q) i /= P.Jl[q];
  return i;
}
__device__ __forceinline__ int kl_index(int k, int l) { return k * (k + 1) / 2 + l; }
// children of region (m-1, pidx) with observations below them, as a bit mask
// (bit c: child c), and the region index of the c-th of them in child order
__device__ __forceinline__ uint32_t active_children(const DevPlan& P, int m, int64_t pidx) {
  uint32_t mask = 0;
  for (int c = 0; c < P.Jl[m]; ++c)
    if (P.slot_post[P.reg_base[m] + pidx * P.Jl[m] + c] >= 0) mask |= 1u << c;
  return mask;
}
__device__ __forceinline__ int64_t nth_child(const DevPlan& P, int m, int64_t pidx, uint32_t mask, int c) {
  for (; c > 0; --c) mask &= mask - 1;
  return pidx * P.Jl[m] + __builtin_ctz(mask);
}
__device__ __forceinline__ int round16(int x) { return x <= 0 ? 0 : ((x + 15) & ~15); }
__device__ __forceinline__ void kl_split(int kl, int& k, int& l) {
  k = 0;
  while ((k + 1) * (k + 2) / 2 <= kl) ++k;
  l = kl - k * (k + 1) / 2;
}

// posterior storage of region (m, i): A^{k,l} tiles, w^k, the inverse
// factor Lt^{-1} of the whitened K~^{-1} = Lt Lt', Z_l = Lt^{-1} A^{m,l},
// z_w = Lt^{-1} w^m, d and u.  Once the forward pass is done the A tiles are
// dead, and the reverse pass keeps its subtree sums there (Grad::Tsum).
struct Post {
  double* base;
  int m;
  __device__ double* A(int k, int l) const { return base + (int64_t)kl_index(k, l) * TT; }
  __device__ double* omega(int k) const { return base + (int64_t)(m + 1) * (m + 2) / 2 * TT + k * T; }
  __device__ double* Lti() const { return base + (int64_t)(m + 1) * (m + 2) / 2 * TT + (m + 1) * T; }
  __device__ double* Z(int l) const { return Lti() + TT + (int64_t)l * TT; }
  __device__ double* zw() const { return Lti() + TT + (int64_t)m * TT; }
  __device__ double* d() const { return zw() + T; }
  __device__ double* u() const { return zw() + T + 1; }
};
__device__ __forceinline__ Post post_of(const DevPlan& P, double* S, int m, int64_t i) {
  Post p;
  p.base = S + P.post_off[m] + (int64_t)P.slot_post[P.reg_base[m] + i] * P.post_stride[m];
  p.m = m;
  return p;
}

__device__ __forceinline__ void record_failure(const DevPlan& P, double* S, int level, int64_t region) {
  atomicCAS((unsigned long long*)(S + P.off_status), 0ull, (unsigned long long)fail_code(level, region));
}

// Row sweep of eq. priorw for 64 rows (points X, nx valid) of a region at
// level `lev` with index `idx`: writes W^^l (l < lev) to rows + l*bstride.
// lds holds LDS_DOUBLES doubles, stage 2 * KC * SLD more (disjoint).
__device__ void row_sweep(const DevPlan& P, double* S, const CovP& c, const double* X, int nx, double* rows,
                          int64_t bstride, int lev, int64_t idx, double* lds, double* stage) {
  Acc acc;
  const int mrows = round16(nx);
  for (int l = 0; l < lev; ++l) {
    const int64_t al = ancestor(P, lev, idx, l);
    const double* Pa = prior_reg(P, S, l, al);
    acc_cov(acc, X, nx, knots_of(P, l, al), P.rl[l], c, false, 0.0);
    gemm_segs2(acc, l, [&](int k) { return seg<Op::N, Op::T>(rows + k * bstride, T, Pa + k * TT, T, -1.0); }, lds,
              mrows);
    double* out = rows + l * bstride;
    // W^^l = W^l L_{a_l}^{-T}: W^l stays in LDS, L^{-1} streams through `stage`
    acc_to_lds(acc, lds);
    __syncthreads();
    acc_zero(acc);
    gemm_lds_a(acc, lds, Pa + (l + 1) * TT, T, false, 1.0, stage, mrows);
    acc_store(acc, out, T);
    __syncthreads();
  }
}


// Blocked left-looking Cholesky of a symmetric nb x nb-tile matrix (tiles
// row-major at base, tile (i, j) at base + (i nb + j) TT, lower tiles read and
// overwritten by the factor), the inverses of its diagonal tiles at dinv,
// and the log-determinant over the first nv rows.  Each tile column takes
// all its updates from the finished columns as one chain of products, then
// its own step.  ok is cleared if a pivot was not positive.
__device__ inline double potrf_tiles(double* base, double* dinv, int nb, int nv, double* lds, double* lds_x,
                                     double* red, bool& ok) {
  double logdet = 0.0;
  Acc acc;
  for (int jb = 0; jb < nb; ++jb) {
    double* Dj = base + ((int64_t)jb * nb + jb) * TT;
    const double* Lj = base + (int64_t)jb * nb * TT;   // row jb of tiles
    acc_load(acc, Dj, T);
    gemm_segs2(acc, jb, [&](int k) { return seg<Op::N, Op::T>(Lj + (int64_t)k * TT, T, Lj + (int64_t)k * TT, T, -1.0); },
              lds);
    acc_to_lds(acc, lds);
    __syncthreads();
    ok = potrf_trtri(lds, lds_x, dinv + (int64_t)jb * TT) && ok;
    logdet += 2.0 * logdiag_lds(lds, min(T, nv - jb * T), red);
    lds_to_global(lds, Dj);
    __syncthreads();
    for (int ib = jb + 1; ib < nb; ++ib) {
      double* X = base + ((int64_t)ib * nb + jb) * TT;
      const double* Li = base + (int64_t)ib * nb * TT;
      acc_load(acc, X, T);
      gemm_segs2(acc, jb,
                [&](int k) { return seg<Op::N, Op::T>(Li + (int64_t)k * TT, T, Lj + (int64_t)k * TT, T, -1.0); }, lds);
      // L_{ib,jb} = (updated tile) L_jb^{-T}: the updated tile stays in LDS,
      // the inverse streams through lds_x (free once the diagonal step is done)
      acc_to_lds(acc, lds);
      __syncthreads();
      acc_zero(acc);
      gemm_lds_a(acc, lds, dinv + (int64_t)jb * TT, T, false, 1.0, lds_x);
      acc_store(acc, X, T);
      __syncthreads();
    }
  }
  return logdet;
}

// reverse-pass storage of region (m, i):
//   G(l), l <= m   cotangent of A^{m,l} of this region (row m of the posterior cotangent)
//   wbar_omega()   cotangent of w^m
//   Wbar(l), l < m cotangent rows of W^^l, then W-bar^l, of the region's knots
//   scratch()      one tile
//   Tsum(l, k)     sum over the subtree's rows of W-bar^l' W^^k, k <= l <= m,
//                  kept in the region's A tiles (dead after the forward pass)
struct Grad {
  double* base;
  double* tbase;   // the region's posterior A tiles
  int m;
  __device__ double* G(int l) const { return base + (int64_t)l * TT; }
  __device__ double* wbar_omega() const { return base + (int64_t)(m + 1) * TT; }
  __device__ double* Wbar(int l) const { return base + (int64_t)(m + 1) * TT + T + (int64_t)l * TT; }
  __device__ double* scratch() const { return base + (int64_t)(m + 1) * TT + T + (int64_t)m * TT; }
  __device__ double* Tsum(int l, int k) const { return tbase + (int64_t)kl_index(l, k) * TT; }
};
__device__ __forceinline__ Grad grad_of(const DevPlan& P, double* S, int m, int64_t i) {
  Grad g;
  const int64_t slot = P.slot_post[P.reg_base[m] + i];
  g.base = S + P.grad_off[m] + slot * P.grad_stride[m];
  g.tbase = S + P.post_off[m] + slot * P.post_stride[m];
  g.m = m;
  return g;
}

}  // namespace mra
