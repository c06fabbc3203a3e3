// Host-side M-RA plan: partition, knots, leaf-sorted padded observations,
// work-arena layout and task lists.  Built without touching the GPU.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mra.h"
#include "devplan.hpp"

namespace mra {

struct GraphCache;  // defined in api.cpp
struct Profiler;    // defined in launch.hpp

// Algorithmic FP64 flops of each launch group for one parameter vector
// (actual r and leaf counts; padding and recomputation are not counted).
struct PhaseFlops {
  double prior[MAXL], post[MAXL], post_reduce[MAXL];
  double leaf_rows, sigma, potrf, trsm, leaf_reduce;
  double rpost[MAXL], rprior[MAXL], rT[MAXL];
  double rleaf_v, rleaf_linv, rleaf_q, rleaf_sbar, rleaf_wbar, rrows, rT_leaf;
  double predict;
};

struct Layout {
  // geometry arena (byte offsets)
  size_t g_knot, g_obs, g_gidx, g_leafn, g_poff, g_soff, g_doff, g_rowt, g_sigt, g_fact, g_trst, g_lint, g_rord;
  size_t g_slotp, g_slotq, g_actp, g_actq;
  size_t g_pxy, g_pgidx, g_pt, g_pleafn, g_ppoff, geom_bytes;
  size_t g_psoff, g_pdoff, g_pcdt, g_pfact;
  // work arena (doubles per theta slice)
  int64_t theta_stride;
};

}  // namespace mra

struct mra_plan_s {
  mra_config cfg;
  int d, M, J, r;
  int64_t n, n_pred;
  std::vector<double> knots;          // r_m x d per region of level m < M, level-major, as built
  std::vector<int64_t> knot_off;      // [M + 1] first entry of level m in knots
  std::vector<int32_t> Jl, rl;        // children per region of level m - 1; knots per region of level m
  std::vector<int64_t> nreg, reg_base;
  std::vector<int64_t> perm;          // leaf order -> original index
  std::vector<int64_t> leaf_off;      // CSR offsets (unpadded)
  std::vector<int32_t> leaf_n;
  std::vector<int64_t> leaf_poff, leaf_soff, leaf_doff;
  int64_t npad = 0, n_sig_tiles = 0, n_dinv_tiles = 0, max_leaf = 0;
  std::vector<double> obs_xy;         // npad x 2
  std::vector<int64_t> obs_gidx;      // npad
  std::vector<double> knot_xy;        // n_internal x T x 2
  // prediction
  std::vector<int64_t> pperm, pleaf_off;
  std::vector<int32_t> pleaf_n;
  std::vector<int64_t> pleaf_poff;
  std::vector<int64_t> pleaf_soff, pleaf_doff;   // remainder-block tiles of each leaf's prediction points
  std::vector<int32_t> pcd_tasks, pfac_tasks;
  int64_t n_pcd_tiles = 0, n_pdinv_tiles = 0;
  int64_t ppad = 0;
  std::vector<double> pred_xy;
  std::vector<int64_t> pred_gidx;
  // task lists
  std::vector<int32_t> row_tasks, sig_tasks, fac_tasks, trsm_tasks, linv_tasks, pred_tasks;
  // fac_tasks are ordered largest leaf first; nbig_thr[t] counts the leaves
  // of >= t tiles, fac_flops_pre / trsm_flops_pre are prefix sums of the
  // algorithmic factorisation and solve flops in that order
  int64_t nbig_thr[16] = {};
  std::vector<double> fac_flops_pre, trsm_flops_pre;
  // tuning: per kernel family launch mapping (mra::Map, 0 = default) and
  // the tile count from which a leaf is factored on the side stream (0: none)
  uint8_t tune[32] = {};
  int32_t big_tiles = 3;
  // reverse-pass leaf solves: on the main stream (0), or on the side stream
  // forked at stage side_solves - 1 of the posterior recursion (ForkHook)
  int32_t side_solves = 2;   // set to M + 2 by build_plan
  // pruning: a region of level m < M is active for the posterior and the
  // reverse pass when observations lie below it, and for the prior when
  // observations or prediction points do; the others get no storage and no
  // task.  slot_*[reg_base[m] + i] is the region's compact index within its
  // level (-1 when pruned); act_* list the active regions level by level
  // (act_*_off[m] .. act_*_off[m + 1]).
  std::vector<int32_t> slot_prior, slot_post, act_prior, act_post;
  std::vector<int64_t> act_prior_off, act_post_off;
  int64_t nact_prior(int m) const { return act_prior_off[m + 1] - act_prior_off[m]; }
  int64_t nact_post(int m) const { return act_post_off[m + 1] - act_post_off[m]; }
  // level-(M-1) regions ordered by their largest child's tile count
  // (ascending, tree order within); nsmall_thr[t] leads with children all
  // below t tiles, whose leaf products need none of the side stream's leaves
  std::vector<int32_t> reduce_order;
  int64_t nsmall_thr[16] = {};
  int64_t nsmall() const { return nsmall_thr[big_tiles < 15 ? big_tiles : 15]; }
  int64_t nbig() const { return big_tiles <= 0 ? 0 : nbig_thr[big_tiles < 15 ? big_tiles : 15]; }
  double potrf_flops_big(int64_t k) const { return fac_flops_pre.empty() ? 0.0 : fac_flops_pre[k]; }
  double trsm_flops_big(int64_t k) const { return trsm_flops_pre.empty() ? 0.0 : trsm_flops_pre[k]; }
  int32_t cut_rrows[9] = {};  // per-XCD chunks of row_tasks balancing the reverse row sweep's cost
  // MRA_CHECKPOINT: the leaf phase runs in nchunks contiguous runs of
  // level-(M-1) regions (one run of all leaves otherwise).  Chunk c holds
  // leaves [chunk_leaf[c], chunk_leaf[c+1]) and padded rows
  // [chunk_row[c], chunk_row[c+1]); every leaf task list is ordered by chunk,
  // and ck_*[c] .. ck_*[c+1] is chunk c's range in it.  The leaf planes hold
  // rows_cap rows (the largest chunk) and L^{-1} ck_soff_cap tiles.
  int32_t nchunks = 1;
  std::vector<int64_t> chunk_leaf, chunk_row, ck_row, ck_sig, ck_fac, ck_linv, ck_red, ck_actq, ck_pred, ck_soff;
  int64_t rows_cap = 0, soff_cap = 0;
  bool checkpoint() const { return (cfg.flags & MRA_CHECKPOINT) != 0; }
  // layout
  mra::Layout lay;
  mra::DevPlan dp;
  bool bound = false;        // geometry and work arena bound
  bool geom_bound = false;   // geometry bound (a work arena may be absent)
  void* d_geom = nullptr;
  void* d_work = nullptr;
  double* call_work = nullptr;   // work arena of the last compute call (status words)
  double flops_loglik = 0, flops_grad = 0, flops_predict = 0;
  // failure of the last synchronised call
  int32_t fail_theta = -1, fail_level = -1;
  int64_t fail_region = -1;
  mra::GraphCache* graphs = nullptr;
  mra::PhaseFlops pf;
  mra::Profiler* prof = nullptr;
  void* side_stream = nullptr;   // hipStream_t for work overlapped with the main stream
  void* ev_fork = nullptr;       // hipEvent_t: main -> side, large leaves' factorisation
  void* ev_big = nullptr;        //   side -> main, large leaves done
  void* ev_fork2 = nullptr;      //   main -> side, reverse-pass leaf solves
  void* ev_join = nullptr;       //   side -> main, V = L^{-T} Y done
  void* ev_join2 = nullptr;      //   side -> main, L^{-1} done
  void* ev_gfork = nullptr;      //   main -> side, the data gather at the start of a call
  void* ev_gath = nullptr;       //   side -> main, data plane written
  int32_t last_nth = 1;
};

namespace mra {
mra_status build_plan(const mra_config* cfg, const double* h_locs, int64_t n, const double* h_pred,
                      int64_t n_pred, const double* h_knots, mra_plan_s* P);
}  // namespace mra
