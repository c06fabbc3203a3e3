// Device-visible description of a bound M-RA plan: pointers into the
// caller's geometry and work arenas plus the level tables.  Passed to every
// kernel by value.
#pragma once
#include <stdint.h>

namespace mra {

constexpr int T = 64;                 // tile edge: knots per region are padded to T
constexpr int64_t TT = (int64_t)T * T;
constexpr int MAXL = 12;              // levels 0..MAXL-1 supported (M <= 11)
constexpr int SIM_DRAWS = 64;         // draws of one mra_simulate call (one tile of columns)

// Failure code written to the per-theta status word: 1 + level * 2^40 + region
__host__ __device__ inline int64_t fail_code(int level, int64_t region) {
  return 1 + ((int64_t)level << 40) + region;
}

struct DevPlan {
  int32_t d, M, cov;
  int32_t Jl[MAXL];          // Jl[m]: children per region of level m - 1 (m = 1..M)
  int32_t rl[MAXL];          // rl[m]: knots per region of level m (m = 0..M-1)
  int64_t n, npad, n_leaves, ppad, n_pred;

  // geometry arena
  const double* knot_xy;     // [n_internal][T][2], padded knots have zero coordinates
  const double* obs_xy;      // [npad][2] leaf-sorted, padded rows zero
  const int64_t* obs_gidx;   // [npad] original index of the row, -1 for padding
  const int32_t* leaf_n;     // [n_leaves] observations per leaf
  const int64_t* leaf_poff;  // [n_leaves + 1] first padded row of each leaf
  const int64_t* leaf_soff;  // [n_leaves] first Sigma tile of each leaf (nb*nb tiles)
  const int64_t* leaf_doff;  // [n_leaves] first diagonal-inverse tile (nb tiles)
  const int32_t* row_tasks;  // [n_row_tasks][2] (leaf, first padded row)
  const int32_t* sig_tasks;  // [n_sig_tasks][3] (leaf, bi, bj), bi >= bj
  const int32_t* fac_tasks;  // [n_fac_tasks] nonempty leaves, largest first
  const int32_t* trsm_tasks; // [n_trsm_tasks][2] (leaf, column plane 0..M)
  const int32_t* linv_tasks; // [n_linv_tasks][2] (leaf, tile column j)
  const int32_t* reduce_order;  // active level-(M-1) regions in leaf-product order
  const int32_t* slot_prior;    // [n_internal] compact prior index within the level, -1 if pruned
  const int32_t* slot_post;     // [n_internal] compact posterior / reverse index, -1 if pruned
  const int32_t* act_prior;     // active regions (prior), level by level
  const int32_t* act_post;      // active regions (posterior and reverse), level by level
  int64_t n_sig_tasks, n_row_tasks;
  int64_t n_sig_tiles;       // leaf-factor tiles (nb * nb per leaf)
  const double* pred_xy;     // [ppad][2]
  const int64_t* pred_gidx;  // [ppad]
  const int32_t* pred_tasks; // [n_pred_tasks][2] (leaf, first padded prediction row)
  const int32_t* pleaf_n;    // [n_leaves]
  const int64_t* pleaf_poff; // [n_leaves + 1]
  // joint predictive distribution (MRA_JOINT): per leaf the first tile of its
  // prediction points' remainder-covariance block (nbp x nbp tiles) and of
  // its diagonal inverses; tasks (leaf, bi, bj), bi >= bj, of those blocks;
  // leaves with prediction points
  const int64_t* pleaf_soff;
  const int64_t* pleaf_doff;
  const int32_t* pcd_tasks;
  const int32_t* pfac_tasks;

  // level tables
  int64_t nreg[MAXL];        // J^m
  int64_t reg_base[MAXL];    // index of the first region of level m among internal regions
  int64_t act_prior_off[MAXL + 1], act_post_off[MAXL + 1];   // level offsets into act_prior / act_post
  int64_t prior_off[MAXL];   // offset (doubles) of level m prior storage in a theta slice
  int64_t post_off[MAXL];    // offset of level m posterior storage
  int64_t post_stride[MAXL]; // doubles per region of level m posterior storage
  int64_t grad_off[MAXL];    // offset of level m reverse-pass storage
  int64_t grad_stride[MAXL];

  // work arena, one slice of theta_stride doubles per parameter vector
  double* work;
  int64_t theta_stride;
  int64_t off_wobs;    // (M+1) planes of [npad][T]; plane M holds z in column 0
  int64_t plane;       // npad * T
  int64_t off_sig;     // Sigma / its Cholesky factor, tiles
  int64_t off_dinv;    // inverses of the diagonal tiles of the leaf factors
  int64_t off_y;       // (M+1) planes: Y = L_Sigma^{-1} [W^ | z]
  int64_t off_leafd;   // [n_leaves] log|Sigma_R|
  int64_t off_status;  // 1 int64 status word
  int64_t off_scal;    // scratch scalars (loglik, partial gradient sums)
  // reverse pass
  int64_t off_v;       // (M+1) planes: V = L_Sigma^{-T} Y
  int64_t off_q;       // (M+1) planes: Q = V Fbar
  int64_t off_sbar;    // Sigma-bar tiles (same layout as off_sig)
  int64_t off_linv;    // tiles of L_Sigma^{-1} (same layout as off_sig)
  int64_t off_wbar;    // M planes: cotangent of the leaf rows of W^ (then W-bar)
  int64_t off_gpart;   // gradient partial sums, [n_gpart][4]: one slot per leaf-factor tile (in leaf
                       // order), per row tile, per internal region; summed in that order, so the
                       // result does not depend on how the tasks are ordered or launched
  int64_t n_gpart;
  // prediction
  int64_t off_pw;      // M planes [ppad][T] of U^ rows, then B~ rows
  int64_t off_pl;      // per prediction tile pl_stride doubles: L^M, then E, tiles
  // generalised least squares (mra_gls): three tiles for the root region (the
  // other regions keep their multi-column quantities in their reverse-pass
  // storage, free until the reverse pass) and a scalar area
  int64_t off_gls0;
  // MRA_JOINT: whitened prior rows U^^k of the prediction points (M planes
  // [ppad][T]), the remainder blocks and their diagonal inverses, the mean in
  // leaf order, and the standard normals of up to SIM_DRAWS draws, each row
  // [n_internal * T region weights | ppad remainder, leaf order]
  int64_t off_pu, off_pcd, off_pdinv, off_pmean, off_sim, n_sim;
  int64_t pl_stride;
};

}  // namespace mra
