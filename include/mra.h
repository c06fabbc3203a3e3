/*
 * mra.h - C ABI of the MI355X multi-resolution approximation (M-RA) library.
 *
 * Computes, for the M-RA of a Gaussian process (Katzfuss, "A multi-resolution
 * approximation for massive spatial datasets", JASA 2017, arXiv 1507.04789):
 *   - the log-likelihood of data z observed with measurement error
 *     (Sec. 3.3 with the leaf covariance of Sec. 4.2),
 *   - its gradient with respect to theta = (log sigma^2, log kappa, log tau^2),
 *   - its gradient with respect to the data,
 *   - the posterior predictive mean and variance of the latent process
 *     (Sec. 3.4, Prop. 2),
 * with all floating point in FP64.
 *
 * Model.  C_0(s, s') = sigma^2 rho(||s - s'|| / kappa), rho the Matern
 * correlation with smoothness 1.5 (eq. mat15) or the exponential
 * correlation exp(-h); data z = y_M(S) + eps, eps ~ N(0, tau^2 I).
 * The domain box is split recursively into J regions per level, levels
 * 0..M (Sec. 2.2); every region below level M holds r knots, the knots of
 * level M are the observations (Sec. 2.2).
 *
 * Memory.  The library never allocates device memory.  mra_requirements
 * reports the byte sizes of a geometry arena and a work arena; the caller
 * allocates them (e.g. as torch tensors) and hands them over in mra_bind.
 * The one exception is the fixed scratch array behind
 * mra_loglik_grad_noalloc (MRA_NOALLOC_MAX_BYTES per GPU, placed by the HIP
 * runtime when the library's code is loaded, never by a call).
 * Pointers named d_* are device pointers owned by the caller; h_* are host
 * pointers owned by the caller and only read during the call.
 *
 * Streams.  Every call that takes a stream enqueues its work on that HIP
 * stream (hipStream_t passed as void*; NULL is the null stream) and returns
 * without waiting unless the plan was built with MRA_SYNC, in which case it
 * synchronises the stream and reports Cholesky breakdowns as MRA_ENOTPD.
 *
 * Ordering.  y, mean and var are in the caller's original order of the
 * locations; the plan permutes internally.
 *
 * Threading.  A plan is not thread-safe; calls on one plan must not overlap.
 */
#ifndef MRA_H
#define MRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mra_plan_s* mra_plan_t;

typedef enum {
  MRA_OK = 0,
  MRA_EINVAL = -1,   /* bad configuration, argument, or location outside the box */
  MRA_ENOTPD = -2,   /* a Cholesky factor broke down (matrix not positive definite) */
  MRA_ENOMEM = -3,   /* host allocation failed or bound arenas too small */
  MRA_EHIP = -4,     /* a HIP runtime call failed */
  MRA_ESTATE = -5    /* call order violated (e.g. loglik before bind) */
} mra_status;

typedef enum { MRA_COV_EXPONENTIAL = 0, MRA_COV_MATERN32 = 1 } mra_cov;

/* flags */
#define MRA_SYNC   1u   /* synchronise after each call and check factor status */
#define MRA_PLAIN  2u   /* one kernel launch per region / task (comparison form) */
#define MRA_GRAPH  4u   /* capture each call's launch sequence in a hipGraph and replay it */
#define MRA_NO_GRAD 8u  /* mra_loglik and mra_predict only: the work arena leaves out the reverse
                           pass's buffers, and mra_loglik_grad(_data) return MRA_ESTATE */
#define MRA_JOINT  32u   /* reserve the buffers of mra_predict_cov and mra_simulate (the joint
                           posterior predictive distribution at the prediction locations) */
#define MRA_CHECKPOINT 16u /* keep the prior blocks (eq. priorw at levels < M) and the leaf
                           factors, and stream the leaf phase through the tree in chunks of
                           level-(M-1) subtrees: the basis rows W^_R of the leaves (the
                           largest blocks of eq. priorw) and their solves exist for one chunk
                           at a time and are recomputed for the reverse pass and kriging
                           instead of being stored for all n; same results to rounding */

/* MRA_GRAPH: the first call with a given (call kind, n_theta, pointer
 * arguments) captures its whole launch sequence, both internal streams
 * included, on a private stream and keeps the instantiated graph; that call
 * and every later call with the same key replays it with one hipGraphLaunch
 * on the caller's stream.  Data behind the pointers (y, theta) is read at
 * replay, so new values in the same buffers need no new capture.  At most
 * 16 graphs are kept (the cache is emptied when a 17th key arrives);
 * mra_bind empties it.  Calls made while profiling is enabled run eagerly. */

typedef struct {
  int32_t d;            /* spatial dimension: 1 or 2 */
  int32_t M;            /* number of partition levels; M = 0 is the exact GP (Sec. 2.4) */
  int32_t J;            /* children per region: d = 2: 1, 2, 4, 8 or 16; d = 1: 1..16 */
  int32_t r;            /* knots per region below level M, 1..64; d = 2 default knots need a square r */
  double lo[2], hi[2];  /* domain box (only the first d entries are read) */
  int32_t cov;          /* mra_cov */
  int32_t max_theta;    /* largest parameter batch a call may pass (>= 1) */
  uint32_t flags;       /* MRA_SYNC | MRA_PLAIN | MRA_GRAPH | MRA_NO_GRAD | MRA_CHECKPOINT | MRA_JOINT */
  int32_t chunks;       /* MRA_CHECKPOINT: leaf chunks (0: 8; at most the level-(M-1) region count) */
  /* Level-dependent partition (Sec. 2.2 with one J per level, as in the
   * satellite application of Sec. 4.2): J_level[m-1] children per region of
   * level m-1 (m = 1..M; 0 = J), r_level[m] knots per region of level m
   * (m = 0..M-1; 0 = r).  d = 2 takes 1, 2, 4, 8 or 16 children per split, a
   * g_x x g_y grid (1x1, 2x1, 2x2, 4x2, 4x4, the larger count along the
   * longer side, x on ties), cut first along y then each slab along x; child
   * iy * g_x + ix.  adaptive = 1 places the split values at quantiles of the
   * observations in the region (then in each slab): t_k = (v[i-1] + v[i]) / 2,
   * v sorted, i = (k * len(v)) / g; fewer than g points fall back to equal
   * parts.  Equal-area split values: a + ((b - a) k) / g, 2-D two-way splits
   * at (a + b) / 2.  Points on a split value go to the upper child. */
  int32_t J_level[12];
  int32_t r_level[12];
  int32_t adaptive;
} mra_config;

typedef struct {
  int64_t n;            /* observations */
  int64_t n_pred;       /* prediction locations */
  int64_t n_rows_pad;   /* observation rows after padding every leaf to a multiple of 64 */
  int64_t n_leaves;     /* J^M */
  int64_t n_regions;    /* sum_m J^m */
  int64_t max_leaf;     /* largest leaf count */
  double flops_loglik;  /* algorithmic FP64 flops of one log-likelihood */
  double flops_grad;    /* algorithmic FP64 flops of one log-likelihood + gradient */
  double flops_predict; /* algorithmic FP64 flops of one prediction pass */
  int64_t n_sim_normals; /* standard normals per draw of mra_simulate: 64 per region below
                            level M (the first r_m used) + n_pred */
} mra_info;

/*
 * Build a plan: partition the box, assign observations and prediction
 * locations to leaves, place knots (Sec. 2.2, 2.5).  Host only; touches no
 * GPU.  h_locs: n x d row-major; h_pred: n_pred x d (may be NULL with
 * n_pred = 0); h_knots: optional explicit knots, r_m x d per region of
 * level m < M in level-major, region-major order, NULL for the default
 * cell-centred grid.  Splits as described at mra_config; d = 2, J = 4: at the midpoint
 * 0.5*(a+b) of each side, child 2*[y >= ymid] + [x >= xmid]; d = 1 at
 * a + ((b-a)*j)/J.  Returns
 * MRA_EINVAL for out-of-box or non-finite locations or unsupported
 * settings, MRA_ENOMEM if a host allocation fails.  *out is owned by the
 * caller and released with mra_destroy.
 */
mra_status mra_build(const mra_config* cfg, const double* h_locs, int64_t n,
                     const double* h_pred, int64_t n_pred, const double* h_knots,
                     mra_plan_t* out);

/* Byte sizes of the geometry arena (theta-independent) and of the work
 * arena (max_theta parameter vectors, all passes).  Host only. */
mra_status mra_requirements(mra_plan_t plan, size_t* geom_bytes, size_t* work_bytes);

/* Sizes and the algorithmic flop counts of the plan.  Host only. */
mra_status mra_get_info(mra_plan_t plan, mra_info* info);

/* Geometry as built, for checking against an independent implementation.
 * Any pointer may be NULL.  h_perm[n]: original index of the k-th
 * observation in leaf order; h_leaf_offsets[J^M + 1]: CSR offsets of the
 * leaves in that order (J_1 ... J_M leaves); h_knots: r_m x d per region of
 * level m < M, level-major.  Host only. */
mra_status mra_get_geometry(mra_plan_t plan, int64_t* h_perm, int64_t* h_leaf_offsets,
                            double* h_knots);

/* Bind caller-owned device arenas (at least the required sizes, 256-byte
 * aligned) and upload the geometry on `stream`.  Must precede every
 * compute call; may be called again to move the plan to new arenas.
 * d_work = NULL with work_bytes = 0 binds the geometry only: then only
 * mra_loglik_grad_noalloc may compute, the other calls return MRA_ESTATE. */
mra_status mra_bind(mra_plan_t plan, void* d_geom, size_t geom_bytes, void* d_work,
                    size_t work_bytes, void* stream);

/*
 * Log-likelihood (Sec. 3.3): loglik = -1/2 (d + u) - (n/2) log(2 pi), with
 * d = log|Sigma|, u = z' Sigma^{-1} z for the M-RA data covariance
 * Sigma(theta) (eq. matrices with m = 0, leaf covariance with tau^2 I).
 * d_y[n] data (original order); d_theta[n_theta][3] = (log sigma^2,
 * log kappa, log tau^2); d_loglik[n_theta] output.  1 <= n_theta <=
 * max_theta.  An entry whose factorisation breaks down is NaN; with
 * MRA_SYNC the call then returns MRA_ENOTPD and mra_last_failure names it.
 */
mra_status mra_loglik(mra_plan_t plan, const double* d_y, const double* d_theta,
                      int32_t n_theta, double* d_loglik, void* stream);

/*
 * Log-likelihood and its gradient d_grad[n_theta][3] =
 * d loglik / d (log sigma^2, log kappa, log tau^2), by a hand-written
 * reverse pass over the prior recursion (eq. priorw), the leaf quantities
 * and the posterior recursion (eq. posterior, helpquantities).
 */
mra_status mra_loglik_grad(mra_plan_t plan, const double* d_y, const double* d_theta,
                           int32_t n_theta, double* d_loglik, double* d_grad, void* stream);

/*
 * As mra_loglik_grad, plus the gradient with respect to the data,
 * d_grad_y[n_theta][n] = d loglik / d z = -Sigma(theta)^{-1} z (caller's
 * order; Sigma as for mra_loglik).  It is the z column of the leaves'
 * bordered-step cotangent in the same reverse pass, so it adds no pass of
 * its own.  Row b of the batch evaluates the data d_y + b * y_stride with
 * the parameters d_theta[b]: y_stride = 0 gives every row the same data,
 * y_stride >= n one data vector per row (several data sets, or one data set
 * with several right-hand sides such as trend columns, in one call).  All
 * outputs are required, in caller-owned device memory that does not overlap
 * d_y.  MRA_EINVAL for a NULL pointer or 0 < y_stride < n, MRA_ESTATE for a
 * plan built with MRA_NO_GRAD.
 */
mra_status mra_loglik_grad_data(mra_plan_t plan, const double* d_y, int64_t y_stride,
                                const double* d_theta, int32_t n_theta, double* d_loglik,
                                double* d_grad, double* d_grad_y, void* stream);

/*
 * Generalised least squares for a linear mean trend z = X beta + (M-RA
 * field with measurement error), at one parameter vector d_theta[3]: the
 * paper states the model for a zero-mean field (Sec. 2.1) and removes the
 * mean before the M-RA (Sec. 4.2); this call estimates a linear mean by
 *   beta = (X' Sigma^{-1} X)^{-1} X' Sigma^{-1} z
 * and returns the profile log-likelihood loglik(z - X beta) (Sec. 3.3) and
 * its gradient in (log sigma^2, log kappa, log tau^2), which, beta
 * maximising the likelihood for every theta, is the gradient at the fixed
 * residual.  One forward pass carries the p trend columns beside z, one
 * reverse pass runs at the residual.
 *   d_y[n]        data (caller's order)
 *   d_X[p][n]     trend columns, column j at d_X + j * n (caller's order), 1 <= p <= 63
 *   d_beta[p]     estimate;  d_loglik[1] profile log-likelihood;  d_grad[3]
 *   d_resid[n]    residual z - X beta (caller's order)
 *   d_XtSiX[p][p] X' Sigma^{-1} X (may be NULL)
 * All device memory owned by the caller; outputs must not overlap inputs.
 * MRA_EINVAL for NULL pointers or p outside 1..63, MRA_ESTATE before
 * mra_bind or for MRA_NO_GRAD plans.  A singular X' Sigma^{-1} X gives NaN
 * outputs and, with MRA_SYNC, MRA_ENOTPD with level M + 1 in
 * mra_last_failure.  Launched eagerly (never captured by MRA_GRAPH).
 */
mra_status mra_gls(mra_plan_t plan, const double* d_y, const double* d_X, int32_t p, const double* d_theta,
                   double* d_beta, double* d_loglik, double* d_grad, double* d_resid, double* d_XtSiX,
                   void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * log-likelihood and gradient as mra_loglik_grad, with the work arena taken
 * from a device array the library owns instead of the bound one.  The call
 * allocates nothing (no hipMalloc, hipFree, stream or event creation; one
 * stream, no captured graph); the caller still owns d_y, d_theta, d_loglik
 * and d_grad.  The plan needs its geometry bound (mra_bind, which accepts
 * d_work = NULL with work_bytes = 0 for this use).
 *
 * Limit: n_theta parameter vectors need n_theta times the per-vector work
 * arena (work_bytes of mra_requirements divided by max_theta), at most
 * MRA_NOALLOC_MAX_BYTES (256 MiB: about three parameter vectors of 4096
 * observations with M = 3, r = 16); larger requests return MRA_ENOMEM
 * before anything is launched.  Each GPU holds one such array from its
 * first use until the process ends; every call on that GPU shares it and
 * leaves its contents behind, so calls that overlap on one GPU (other
 * streams, other plans, other threads) race and must be serialised by the
 * caller.  MRA_EINVAL for NULL pointers or n_theta outside 1..max_theta,
 * MRA_ESTATE before mra_bind or for a plan built with MRA_NO_GRAD.
 */
#define MRA_NOALLOC_MAX_BYTES ((size_t)256 << 20)
mra_status mra_loglik_grad_noalloc(mra_plan_t plan, const double* d_y, const double* d_theta,
                                   int32_t n_theta, double* d_loglik, double* d_grad, void* stream);

/*
 * Posterior predictive mean and variance of the latent process y_M at the
 * plan's prediction locations (Prop. 2, marginal variances), for one
 * parameter vector d_theta[3].  d_mean[n_pred], d_var[n_pred] in the
 * original order of h_pred.
 */
mra_status mra_predict(mra_plan_t plan, const double* d_y, const double* d_theta,
                       double* d_mean, double* d_var, void* stream);

/*
 * Joint posterior predictive distribution (Prop. 2 and the remark after
 * it): the posterior predictive of y_M at the prediction locations has the
 * M-RA form sum_{m<M} B~^{m+1,m} eta~_{a_m} + delta~ with independent region
 * weights eta~ ~ N(K~ w^m, K~) and leaf remainders delta~ ~ N(L^M Sigma^{-1}
 * z_R, V^P - L^M Sigma^{-1} L^M'), so its covariance is the sum over shared
 * regions of B~ K~ B~' plus, within a leaf, the remainder block.  Plans need
 * MRA_JOINT (otherwise MRA_ESTATE); one parameter vector d_theta[3].
 *
 * mra_predict_cov: d_mean[n_pred] and the dense covariance matrix
 * d_cov[n_pred][n_pred] (row-major, caller's order of h_pred).
 *
 * mra_simulate: n_draws (1..MRA_SIM_MAX_DRAWS) conditional draws of y_M at
 * the prediction locations, d_out[n_draws][n_pred], from caller-supplied
 * standard normals d_eps[n_draws][eps_stride], eps_stride >= n_sim_normals
 * of mra_get_info: row d holds 64 normals per region below level M in
 * level-major, region-major order ((N_m + i) * 64 for region (m, i), N_m
 * the number of regions above level m, i.e. sum_{l<m} J_1 ... J_l; the
 * first r_m of the 64 are used) followed by one normal per prediction
 * location in the caller's order.  Draw d is
 *   mean + sum_m B~^{m+1,m} Lt_{a_m}^{-T} xi_{a_m} + chol(remainder block) xi_R
 * (Lt Lt' the whitened K~^{-1}), a linear function of the normals.  The
 * prediction locations of a leaf must be distinct (the remainder block is
 * factored; MRA_ENOTPD otherwise).
 */
#define MRA_SIM_MAX_DRAWS 64
mra_status mra_predict_cov(mra_plan_t plan, const double* d_y, const double* d_theta, double* d_mean,
                           double* d_cov, void* stream);
mra_status mra_simulate(mra_plan_t plan, const double* d_y, const double* d_theta, const double* d_eps,
                        int64_t eps_stride, int32_t n_draws, double* d_out, void* stream);

/* After a call that returned MRA_ENOTPD (or after synchronising a call
 * made without MRA_SYNC): the first failing (theta index, level, region).
 * Synchronises `stream`.  Returns MRA_OK with theta_idx = -1 if none. */
mra_status mra_last_failure(mra_plan_t plan, int32_t* theta_idx, int32_t* level,
                            int64_t* region, void* stream);

/*
 * Autotuner.  Every batched launch belongs to a kernel family (prior,
 * leaf_rows, leaf_sigma, leaf_potrf, leaf_trsm, leaf_reduce, post,
 * post_reduce, rleaf_v, rleaf_linv, rpost, rleaf_q, rleaf_sbar, rrows_leaf,
 * rT_leaf, rprior, rT, predict).  A family's launch shape is the mapping of
 * workgroups to its tasks: "identity", "grouped" (related tasks, e.g. the
 * planes of one leaf, on one XCD and L2) or "chunked" (one contiguous run of
 * the tree-ordered task list per XCD); "default" keeps the built-in choice.
 * big_leaf_tiles is the tile count from which a leaf is factored on the
 * second stream (0: none).  side_solves places the reverse pass's leaf
 * solves: 0 on the main stream; s >= 1 on the second stream, forked once the
 * recursion has reached stage s - 1 (0: before the leaf reduction, 1: after
 * it, 1 + j: after posterior level M - j, M + 2 + m: after the reverse
 * posterior step of level m; larger values fork after the last of those), so
 * that they fill the GPU while the coarse levels' latency-bound steps run.
 * Shapes only permute work: results are the same bit for bit under every
 * table.
 *
 * mra_autotune times mra_loglik_grad (mra_loglik for MRA_NO_GRAD plans) on
 * the given device data, `reps` calls per candidate after one warm-up call,
 * over one pass of coordinate descent (each family's shapes, then the leaf
 * cut), keeps the fastest table, and writes it as JSON to out_json (cap
 * bytes; *len receives the length, without the terminating zero; MRA_ENOMEM
 * if cap is too small, the table is applied anyway).  d_loglik [n_theta] and
 * d_grad [n_theta][3] are scratch outputs.  Synchronises `stream`.
 * mra_get_tuning writes the current table; mra_set_tuning applies a table
 * produced by either: unknown keys are ignored, families the table omits
 * take their built-in shape, an omitted big_leaf_tiles or side_solves keeps
 * its value; an unknown shape, a malformed value or an integer outside
 * 0..64 gives MRA_EINVAL and leaves the table unchanged.  mra_set_tuning
 * and mra_autotune drop captured graphs.  Host only apart from
 * mra_autotune.
 */
mra_status mra_autotune(mra_plan_t plan, const double* d_y, const double* d_theta, int32_t n_theta,
                        double* d_loglik, double* d_grad, int32_t reps, char* out_json, size_t cap,
                        size_t* len, void* stream);
mra_status mra_get_tuning(mra_plan_t plan, char* out_json, size_t cap, size_t* len);
mra_status mra_set_tuning(mra_plan_t plan, const char* json);

/* Per-kernel timing (tracing).  mra_profile(plan, 1) enables HIP-event
 * timing of every launch group of the following calls on their streams and
 * clears earlier records; mra_profile(plan, 0) disables it.
 * mra_profile_read synchronises `stream`, aggregates the records by
 * (kernel, level) into out[0..cap), sets *count to the number of distinct
 * entries (which may exceed cap) and clears the records. */
typedef struct {
  char name[24];      /* kernel family, e.g. "leaf_reduce" */
  int32_t level;      /* tree level for per-level kernels, -1 otherwise */
  int64_t groups;     /* timed launch groups */
  int64_t launches;   /* kernel launches (one per task in the plain form) */
  double total_ms;    /* summed event time of the groups */
  double flops;       /* summed algorithmic FP64 flops of the groups */
} mra_phase_stat;

mra_status mra_profile(mra_plan_t plan, int32_t enable);
mra_status mra_profile_read(mra_plan_t plan, mra_phase_stat* out, int32_t cap, int32_t* count, void* stream);

const char* mra_status_string(mra_status s);

/* Release the plan (and any captured graphs).  Does not free the arenas. */
void mra_destroy(mra_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* MRA_H */
