// Generalised least squares for a linear mean trend (mra_gls).
//
// The model of Sec. 2.1 is written for a zero-mean field; a trend X beta
// is removed before the M-RA (Sec. 4.2 removes the mean of the satellite
// data).  With the M-RA data covariance Sigma (eq. matrices, leaf
// covariance with tau^2 I) the generalised least-squares estimate is
//   beta = (X' Sigma^{-1} X)^{-1} X' Sigma^{-1} z,
// the profile log-likelihood is loglik(z - X beta) and, beta maximising the
// likelihood for every theta, its gradient is the gradient at the fixed
// residual r = z - X beta.
//
// One pass.  The trend columns ride in the spare columns 1..p of the data
// plane beside z (column 0), so the leaf solves Y = L_Sigma^{-1} [W^ | z X]
// of the ordinary forward pass already hold Sigma_R^{-1}-solves of every
// column.  The posterior recursion (eq. posterior, helpquantities) is then
// repeated for the R = 1 + p data columns at once, reusing the stored
// posterior factors (whitened: Lt^{-1}, Z_l = Lt^{-1} A^{m,l}):
//   leaves:  Omega^k = sum_c Y^k_c' Y^z_c (k < M),  U = sum_c Y^z_c' Y^z_c,
//   region:  zW = Lt^{-1} Omega^m,  U -= zW' zW,
//   parent:  Omega^k_P = sum_c (Omega^k_c - Z^k_c' zW_c),  U_P = sum_c U_c,
// the column-wise form of the omega~ and u recursions of Sec. 3.3, so that
// the root's U = [z X]' Sigma^{-1} [z X].  beta and the profile u follow
// from U; omega and z_w are linear in the data, so the residual's z_w at
// every region and its leaf solve L_Sigma^{-1} r are linear combinations
// of the stored columns, and the ordinary reverse pass then gives the
// gradient at r.
#include "common.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace mra {

// multi-column storage of region (m, i): Omega^0..Omega^m, zW, U (tiles
// 0..m, m+1, m+2).  The reverse pass's storage of the region is free until
// the reverse pass starts (m >= 1 holds 2m + 2 >= m + 3 tiles); the root
// uses tiles of its own.
__device__ __forceinline__ double* gls_of(const DevPlan& P, double* S, int m, int64_t i) {
  if (m == 0) return S + P.off_gls0;
  return grad_of(P, S, m, i).base;
}

// level-(M-1) regions, task (q, k): Omega^k (k < M) or U (k = M) summed over
// the region's leaves, R data columns
__global__ __launch_bounds__(NT) void k_gls_leaf(DevPlan P, int R, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int M = P.M;
  const int64_t pidx = P.reduce_order[tk0 / (M + 1)];
  const int k = (int)(tk0 % (M + 1));
  double* S = slice(P, 0);
  double* G = gls_of(P, S, M - 1, pidx);
  const double* Yk = S + P.off_y + (int64_t)k * P.plane;
  const double* Yz = S + P.off_y + (int64_t)M * P.plane;
  const int JM = P.Jl[M];
  int nsg = 0;
  for (int c = 0; c < JM; ++c) {
    const int64_t leaf = pidx * JM + c;
    nsg += (int)((P.leaf_poff[leaf + 1] - P.leaf_poff[leaf]) / T);
  }
  Acc acc;
  acc_zero(acc);
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
    return seg<Op::T, Op::N>(Yk + p * T, T, Yz + p * T, T, 1.0, round16(rows) / KC);
  }, lds, k == M ? round16(R) : T, round16(R));
  acc_store(acc, G + (int64_t)(k < M ? k : M + 1) * TT, T);
}

// M = 0: U = Y' Y over the single leaf
__global__ __launch_bounds__(NT) void k_gls_root_leaf(DevPlan P, int R) {
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  double* S = slice(P, 0);
  const double* Yz = S + P.off_y;
  const int nsg = (int)((P.leaf_poff[1] - P.leaf_poff[0]) / T);
  Acc acc;
  acc_zero(acc);
  gemm_segs2(acc, nsg, [&](int sg) {
    const int64_t p = (int64_t)sg * T;
    return seg<Op::T, Op::N>(Yz + p * T, T, Yz + p * T, T, 1.0, round16(min(T, P.leaf_n[0] - T * sg)) / KC);
  }, lds, round16(R), round16(R));
  acc_store(acc, S + P.off_gls0 + 2 * TT, T);
}

// region of level m: zW = Lt^{-1} Omega^m, U -= zW' zW
__global__ __launch_bounds__(NT) void k_gls_post(DevPlan P, int m, int R, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int64_t i = P.act_post[P.act_post_off[m] + tk0];
  double* S = slice(P, 0);
  const Post po = post_of(P, S, m, i);
  double* G = gls_of(P, S, m, i);
  double* zW = G + (int64_t)(m + 1) * TT;
  double* U = G + (int64_t)(m + 2) * TT;
  const int rc = round16(R);
  Acc acc;
  acc_zero(acc);
  gemm_segs(acc, 1, [&](int) { return seg<Op::N, Op::N>(po.Lti(), T, G + (int64_t)m * TT, T, 1.0); }, lds, T, rc);
  acc_store(acc, zW, T);
  __syncthreads();
  acc_load(acc, U, T);
  gemm_segs(acc, 1, [&](int) { return seg<Op::T, Op::N>(zW, T, zW, T, -1.0); }, lds, rc, rc);
  acc_store(acc, U, T);
}

// parent of level m - 1, task (q, k): Omega^k_P = sum_c (Omega^k_c - Z^k_c' zW_c)
// for k < m, U_P = sum_c U_c for k = m (children with observations below them)
__global__ __launch_bounds__(NT) void k_gls_reduce(DevPlan P, int m, int R, TaskMap tm) {
  const int64_t tk0 = task_of(tm);
  if (tk0 < 0) return;
  __shared__ __attribute__((aligned(32))) double lds[LDS_DOUBLES];
  const int64_t pidx = P.act_post[P.act_post_off[m - 1] + tk0 / (m + 1)];
  const int k = (int)(tk0 % (m + 1));
  double* S = slice(P, 0);
  int64_t ch[16];
  int nch = 0;
  for (int c = 0; c < P.Jl[m]; ++c)
    if (post_active(P, m, pidx * P.Jl[m] + c)) ch[nch++] = pidx * P.Jl[m] + c;
  double* GP = gls_of(P, S, m - 1, pidx);
  Acc acc;
  acc_zero(acc);
  if (k == m) {
    for (int c = 0; c < nch; ++c) acc_load(acc, gls_of(P, S, m, ch[c]) + (int64_t)(m + 2) * TT, T, true);
    acc_store(acc, GP + (int64_t)(m + 1) * TT, T);
    return;
  }
  for (int c = 0; c < nch; ++c) acc_load(acc, gls_of(P, S, m, ch[c]) + (int64_t)k * TT, T, true);
  gemm_segs2(acc, nch, [&](int c) {
    const Post pc = post_of(P, S, m, ch[c]);
    return seg<Op::T, Op::N>(pc.Z(k), T, gls_of(P, S, m, ch[c]) + (int64_t)(m + 1) * TT, T, -1.0);
  }, lds, T, round16(R));
  acc_store(acc, GP + (int64_t)k * TT, T);
}

// root: the p x p normal equations X' Sigma^{-1} X beta = X' Sigma^{-1} z by a
// Cholesky solve in LDS (one thread; p <= 63), the profile quadratic form
// u_r = z' Sigma^{-1} z - beta' X' Sigma^{-1} z and the profile
// log-likelihood -1/2 (d + u_r) - (n/2) log 2 pi
__global__ __launch_bounds__(64) void k_gls_solve(DevPlan P, int R, double* beta, double* out_ll, double* xtsix) {
  __shared__ double A[T * T];
  __shared__ double b[T];
  double* S = slice(P, 0);
  const double* U = (P.M > 0 ? gls_of(P, S, 0, 0) : S + P.off_gls0) + 2 * TT;
  const int p = R - 1;
  for (int e = threadIdx.x; e < p * p; e += 64) {
    const int i = e / p, j = e % p;
    A[i * T + j] = U[(1 + i) * T + 1 + j];
    if (xtsix) xtsix[e] = A[i * T + j];
  }
  for (int i = threadIdx.x; i < p; i += 64) b[i] = U[(1 + i) * T];
  __syncthreads();
  if (threadIdx.x != 0) return;
  bool ok = true;
  for (int j = 0; j < p; ++j) {       // A = L L' in place (lower triangle)
    double a = A[j * T + j];
    for (int k = 0; k < j; ++k) a -= A[j * T + k] * A[j * T + k];
    if (!(a > 0.0)) ok = false;
    const double d = sqrt(a);
    A[j * T + j] = d;
    for (int i = j + 1; i < p; ++i) {
      double s = A[i * T + j];
      for (int k = 0; k < j; ++k) s -= A[i * T + k] * A[j * T + k];
      A[i * T + j] = s / d;
    }
  }
  double x[T];
  for (int i = 0; i < p; ++i) {       // L y = b
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= A[i * T + k] * x[k];
    x[i] = s / A[i * T + i];
  }
  for (int i = p - 1; i >= 0; --i) {  // L' beta = y
    double s = x[i];
    for (int k = i + 1; k < p; ++k) s -= A[k * T + i] * x[k];
    x[i] = s / A[i * T + i];
  }
  double bx = 0.0;
  for (int i = 0; i < p; ++i) bx += b[i] * x[i];
  const double d = P.M > 0 ? *post_of(P, S, 0, 0).d() : S[P.off_leafd];
  const double nan = __builtin_nan("");
  const double ll = -0.5 * (d + (U[0] - bx)) - 0.5 * (double)P.n * 1.8378770664093453;
  if (!ok) record_failure(P, S, P.M + 1, 0);
  for (int i = 0; i < p; ++i) beta[i] = ok ? x[i] : nan;
  *out_ll = ok ? ll : nan;
}

// residual r = z - X beta in the caller's order
__global__ void k_gls_resid(const double* y, const double* X, int p, int64_t n, const double* beta, double* resid) {
  for (int64_t g = blockIdx.x * (int64_t)NT + threadIdx.x; g < n; g += (int64_t)gridDim.x * NT) {
    double r = y[g];
    for (int j = 0; j < p; ++j) r -= beta[j] * X[(int64_t)j * n + g];
    resid[g] = r;
  }
}

// leaf planes of the residual (one plane set for all leaves): the data
// plane's column 0 becomes r and the solve's column 0 becomes
// L_Sigma^{-1} r = Y^z_0 - sum_j beta_j Y^z_{1+j}; the trend columns are cleared
__global__ void k_gls_planes(DevPlan P, const double* resid, int p, const double* beta) {
  double* S = slice(P, 0);
  double* zp = S + P.off_wobs + (int64_t)P.M * P.plane;
  double* yz = S + P.off_y + (int64_t)P.M * P.plane;
  for (int64_t q = blockIdx.x * (int64_t)NT + threadIdx.x; q < P.npad; q += (int64_t)gridDim.x * NT) {
    const int64_t g = P.obs_gidx[q];
    double y0 = yz[q * T];
    for (int j = 0; j < p; ++j) {
      y0 -= beta[j] * yz[q * T + 1 + j];
      yz[q * T + 1 + j] = 0.0;
      zp[q * T + 1 + j] = 0.0;
    }
    yz[q * T] = y0;
    zp[q * T] = g >= 0 ? resid[g] : 0.0;
  }
}

// regions of level m: z_w of the residual, zW_0 - sum_j beta_j zW_{1+j}
__global__ void k_gls_regions(DevPlan P, int m, int p, const double* beta) {
  double* S = slice(P, 0);
  const int64_t i = P.act_post[P.act_post_off[m] + blockIdx.x];
  const double* zW = gls_of(P, S, m, i) + (int64_t)(m + 1) * TT;
  double* zw = post_of(P, S, m, i).zw();
  const int r = threadIdx.x;
  double v = zW[r * T];
  for (int j = 0; j < p; ++j) v -= beta[j] * zW[r * T + 1 + j];
  zw[r] = v;
}

// the level-(M-1) products of the reduce-order regions [q0, q1)
hipError_t launch_gls_leaf(const mra_plan_s& H, const DevPlan& P, int64_t q0, int64_t q1, int R, hipStream_t st) {
  Runner run{P, 1, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  const int M = P.M;
  const int64_t nq = (int64_t)H.reduce_order.size();
  double rs = 0.0;
  for (int l = 0; l < M; ++l) rs += P.rl[l];
  const double f = nq > 0 ? 2.0 * (double)P.n * (rs + R) * R * (double)(q1 - q0) / (double)nq : 0.0;
  run.range("gls_leaf", -1, f, M + 1, k_gls_leaf, q0 * (M + 1), q1 * (M + 1), R);
  return hipGetLastError();
}

// The whole GLS call for one parameter vector: forward pass with the trend
// columns beside the data, the multi-column posterior, the normal
// equations, the residual's forward quantities and the reverse pass at the
// residual.  No second stream.
hipError_t launch_gls(const mra_plan_s& H, const double* y, const double* X, int p, const double* theta, double* beta,
                      double* out_ll, double* xtsix, double* grad, double* resid, hipStream_t st) {
  const DevPlan& P = H.dp;
  const int M = P.M;
  const int R = p + 1;
  hipError_t e;
  if ((e = launch_forward_front(H, y, theta, 1, st, nullptr, 0, X, p)) != hipSuccess) return e;
  if ((e = launch_forward_back(H, 1, nullptr, st, nullptr, nullptr)) != hipSuccess) return e;
  Runner run{P, 1, st, (H.cfg.flags & MRA_PLAIN) != 0, H.prof, H.tune};
  if (M == 0) {
    hipLaunchKernelGGL(k_gls_root_leaf, dim3(1), dim3(NT), 0, st, P, R);
  } else {
    if (H.nchunks == 1 && (e = launch_gls_leaf(H, P, 0, (int64_t)H.reduce_order.size(), R, st)) != hipSuccess)
      return e;   // with MRA_CHECKPOINT these ran chunk by chunk in the forward pass
    for (int m = M - 1; m >= 0; --m) {
      run.range("gls_post", m, 0.0, 1, k_gls_post, 0, H.nact_post(m), m, R);
      if (m > 0) run.range("gls_reduce", m, 0.0, m + 1, k_gls_reduce, 0, H.nact_post(m - 1) * (int64_t)(m + 1), m, R);
    }
  }
  hipLaunchKernelGGL(k_gls_solve, dim3(1), dim3(64), 0, st, P, R, beta, out_ll, xtsix);
  int64_t gx = (P.n + NT - 1) / NT;
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_gls_resid, dim3((unsigned)gx), dim3(NT), 0, st, y, X, p, P.n, beta, resid);
  if (H.nchunks == 1) {
    int64_t gp = (P.npad + NT - 1) / NT;
    if (gp > 4096) gp = 4096;
    hipLaunchKernelGGL(k_gls_planes, dim3((unsigned)gp), dim3(NT), 0, st, P, resid, p, beta);
  }
  for (int m = 0; m < M; ++m)
    if (H.nact_post(m) > 0)
      hipLaunchKernelGGL(k_gls_regions, dim3((unsigned)H.nact_post(m)), dim3(T), 0, st, P, m, p, beta);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the reverse pass at the residual (with MRA_CHECKPOINT the leaf planes are
  // recomputed from `resid`)
  if ((e = launch_grad_leafsolve(H, 1, st)) != hipSuccess) return e;
  if ((e = launch_grad_post(H, 1, st, nullptr)) != hipSuccess) return e;
  return launch_grad_rest(H, resid, 0, theta, 1, grad, nullptr, st, nullptr);
}

}  // namespace mra
