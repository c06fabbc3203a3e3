// Launch helper shared by the kernel files: a batch of independent tasks is
// one launch (grid.x = tasks, grid.y = parameter vectors), or, in the plain
// comparison form, one launch per task.  With profiling enabled every launch
// group is bracketed by HIP events on the call's stream.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "devplan.hpp"

struct mra_plan_s;

namespace mra {

// Task index of a workgroup.  Workgroups are dispatched to the 8 XCDs
// round-robin by block index, so block b runs on XCD b % 8, and each XCD has
// its own L2.  Batched launches of tasks that share inputs (G consecutive
// task indices) place each group on one XCD: group g goes to XCD g % 8, and
// its G tasks take consecutive slots there, so they find the group's inputs
// in that XCD's L2.  G = 0 gives XCD x the contiguous chunk
// [cut[x], cut[x+1]) of the task list, walked in order: tasks in tree order
// that share ancestors run close together in time on one XCD.  The cuts
// balance the chunks' estimated cost.  Blocks past the last task of their
// group or chunk return -1.
struct TaskMap {
  int64_t t0;       // first task (plain form: the single task of the launch)
  int64_t ntask;    // tasks in the launch (a multiple of G when G > 1)
  int32_t G;        // group size; 1 = identity mapping, 0 = one chunk per XCD
  int32_t cut[9];   // G = 0: chunk boundaries, cut[0] = 0, cut[8] = ntask
};

__device__ __forceinline__ int64_t task_of(const TaskMap& m) {
  const int64_t b = blockIdx.x;
  if (m.G == 1) return m.t0 + b;
  if (m.G == 0) {
    const int x = (int)(b & 7);
    const int64_t t = m.cut[x] + (b >> 3);
    return t < m.cut[x + 1] ? m.t0 + t : -1;
  }
  const int64_t xcd = b & 7, s = b >> 3;
  const int64_t g = (s / m.G) * 8 + xcd;
  if (g * m.G >= m.ntask) return -1;
  return m.t0 + g * m.G + (s % m.G);
}

// Tunable launch shapes.  Every batched launch belongs to a kernel family;
// the plan's table picks, per family, how workgroups map to tasks (identity,
// groups of related tasks on one XCD, or one contiguous chunk per XCD).  The
// mapping only permutes tasks over workgroups, so results do not depend on it.
enum Fam : int {
  F_PRIOR, F_LEAF_ROWS, F_SIGMA, F_POTRF, F_TRSM, F_LEAF_REDUCE, F_POST, F_POST_REDUCE, F_RLEAF_V, F_RLEAF_LINV,
  F_RPOST, F_RLEAF_Q, F_RLEAF_SBAR, F_RROWS, F_RT_LEAF, F_RPRIOR, F_RT, F_PREDICT, F_COUNT
};
enum Map : uint8_t { MAP_DEFAULT = 0, MAP_IDENTITY = 1, MAP_GROUPED = 2, MAP_CHUNKED = 3 };
inline const char* fam_name(int f) {
  static const char* n[F_COUNT] = {"prior", "leaf_rows", "leaf_sigma", "leaf_potrf", "leaf_trsm", "leaf_reduce",
                                   "post", "post_reduce", "rleaf_v", "rleaf_linv", "rpost", "rleaf_q", "rleaf_sbar",
                                   "rrows_leaf", "rT_leaf", "rprior", "rT", "predict"};
  return (f >= 0 && f < F_COUNT) ? n[f] : "";
}
inline const char* map_name(int m) {
  static const char* n[4] = {"default", "identity", "grouped", "chunked"};
  return (m >= 0 && m < 4) ? n[m] : "";
}

struct ProfRecord {
  const char* name;
  int level;
  double flops;          // algorithmic flops of the group (all parameter vectors)
  int64_t launches;
  hipEvent_t start, stop;
};

struct Profiler {
  bool enabled = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRecord> recs;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct Runner {
  const DevPlan& P;
  int nth;
  hipStream_t st;
  bool plain;
  Profiler* prof;
  const uint8_t* tune = nullptr;   // F_COUNT entries of Map, or null for the defaults
  // tasks [t_begin, t_end) of family f: the table's mapping, else dflt;
  // G is the family's natural group size, cut its chunk boundaries (or null)
  template <class K, class... A>
  void tuned(Fam f, Map dflt, const char* name, int level, double flops, int G, const int32_t* cut, K kern,
             int64_t t_begin, int64_t t_end, A... args) const {
    Map m = (tune && tune[f] != MAP_DEFAULT) ? (Map)tune[f] : dflt;
    if (m == MAP_GROUPED && G <= 1) m = MAP_IDENTITY;
    if (m == MAP_CHUNKED) {
      chunked_range(name, level, flops, t_begin == 0 ? cut : nullptr, kern, t_begin, t_end, args...);
    } else {
      range(name, level, flops, m == MAP_GROUPED ? G : 1, kern, t_begin, t_end, args...);
    }
  }
  template <class K, class... A>
  void operator()(const char* name, int level, double flops, K kern, int64_t ntask, A... args) const {
    grouped(name, level, flops, 1, kern, ntask, args...);
  }
  // tasks [t_begin, t_end) in one contiguous chunk per XCD (G = 0), cut at
  // `cut` (relative to t_begin; equal task counts when null)
  template <class K, class... A>
  void chunked_range(const char* name, int level, double flops, const int32_t* cut, K kern, int64_t t_begin,
                     int64_t t_end, A... args) const {
    const int64_t ntask = t_end - t_begin;
    if (ntask <= 0) return;
    TaskMap tm{t_begin, ntask, 0, {}};
    int64_t widest = 0;
    for (int x = 0; x <= 8; ++x) tm.cut[x] = cut ? cut[x] : (int32_t)(ntask * x / 8);
    for (int x = 0; x < 8; ++x) widest = std::max<int64_t>(widest, tm.cut[x + 1] - tm.cut[x]);
    launch(name, level, flops, kern, ntask, dim3((unsigned)(8 * widest), nth), tm, args...);
  }
  template <class K, class... A>
  void grouped(const char* name, int level, double flops, int G, K kern, int64_t ntask, A... args) const {
    range(name, level, flops, G, kern, 0, ntask, args...);
  }
  // tasks [t_begin, t_end) of a task list
  template <class K, class... A>
  void range(const char* name, int level, double flops, int G, K kern, int64_t t_begin, int64_t t_end, A... args) const {
    const int64_t ntask = t_end - t_begin;
    if (ntask <= 0) return;
    if (G == 1) {
      launch(name, level, flops, kern, ntask, dim3((unsigned)ntask, nth), TaskMap{t_begin, ntask, 1, {}}, args...);
    } else {
      const int64_t ngroups = ntask / G;
      const int64_t nblk = (ngroups + 7) / 8 * 8 * G;
      launch(name, level, flops, kern, ntask, dim3((unsigned)nblk, nth), TaskMap{t_begin, ntask, G, {}}, args...);
    }
  }
  // one batched launch of `grid` blocks with mapping tm, or in the plain form
  // one launch per task
  template <class K, class... A>
  void launch(const char* name, int level, double flops, K kern, int64_t ntask, dim3 grid, const TaskMap& tm,
              A... args) const {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof && prof->enabled) {
      e0 = prof->next();
      e1 = prof->next();
      if (e0) (void)hipEventRecord(e0, st);
    }
    if (plain) {
      for (int64_t t = tm.t0; t < tm.t0 + ntask; ++t)
        hipLaunchKernelGGL(kern, dim3(1, nth), dim3(256), 0, st, P, args..., TaskMap{t, 1, 1, {}});
    } else {
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, P, args..., tm);
    }
    if (e0 && e1) {
      (void)hipEventRecord(e1, st);
      prof->recs.push_back(ProfRecord{name, level, flops * nth, plain ? ntask : 1, e0, e1});
    }
  }
};

hipError_t launch_forward(const mra_plan_s& H, const double* y, const double* theta, int nth, double* out_loglik,
                          hipStream_t st);
// A second stream for work that only needs the leaf factors.  Large leaves
// (big_tiles tiles or more) are factored on it, forked after the Sigma
// tiles (fork) and awaited by the main stream before the leaf products of
// their parents (big); the reverse pass's leaf solves follow on it (fork2,
// join).  A null Side runs everything on the main stream.
struct Side {
  hipStream_t s;
  hipEvent_t fork, big, fork2, join, join2;   // join: V done; join2: L^{-1} done
  hipEvent_t gfork, gath;                     // the data gather, forked at the start of a call
};
// y_stride: parameter row b uses the data y + b * y_stride (0: the same data for all rows)
// X (may be null): p trend columns [p][n] (caller's order) carried beside the
// data in columns 1..p of the data plane (generalised least squares)
hipError_t launch_forward_front(const mra_plan_s& H, const double* y, const double* theta, int nth, hipStream_t st,
                                const Side* side = nullptr, int64_t y_stride = 0, const double* X = nullptr,
                                int px = 0);
// A callback run once, when the launches of its stage have been enqueued on
// the main stream: 0 before the leaf reduction, 1 after it, 1 + j after
// posterior level M - j (and its child sums), j = 1..M, then M + 2 + m after
// the reverse posterior step of level m, m = 0..M-1; a later stage runs at
// the end of the reverse posterior.  Used to fork independent work onto the
// side stream at a chosen point of the recursion.
struct ForkHook {
  int stage;
  hipError_t (*fn)(void* ctx);
  void* ctx;
  bool fired;
  hipError_t at(int s, bool last = false) {
    if (fired || (!last && s < stage)) return hipSuccess;
    fired = true;
    return fn(ctx);
  }
};
hipError_t launch_forward_back(const mra_plan_s& H, int nth, double* out_loglik, hipStream_t st,
                               const Side* side = nullptr, ForkHook* hook = nullptr);
// after_v (may be null) is recorded on st once V is written, before L^{-1}
hipError_t launch_grad_leafsolve(const mra_plan_s& H, int nth, hipStream_t st, hipEvent_t after_v = nullptr);
hipError_t launch_zero_gpart(const mra_plan_s& H, int nth, hipStream_t st);
hipError_t launch_grad_post(const mra_plan_s& H, int nth, hipStream_t st, ForkHook* hook = nullptr,
                            bool zero_partials = true);
// grad_y (may be null): [nth][n] gradient of the log-likelihood with respect
// to the data, in the caller's order
// wait_linv (may be null): event to wait for before the first use of L^{-1}
hipError_t launch_grad_rest(const mra_plan_s& H, const double* y, int64_t y_stride, const double* theta, int nth,
                            double* out_grad, double* grad_y, hipStream_t st, hipEvent_t wait_linv = nullptr);
// MRA_CHECKPOINT leaf chunks: the device plan of chunk c (plane and L^{-1}
// offsets shifted to the chunk's buffers; the whole plan for one chunk), and
// the chunk's leaf planes (data, W^, Y; with factor also Sigma and its
// factor, otherwise recomputed from the stored factors)
DevPlan chunk_plan(const mra_plan_s& H, int c);
hipError_t launch_leaf_planes(const mra_plan_s& H, int c, const double* y, const double* theta, int nth,
                              hipStream_t st, int64_t y_stride, bool factor, const double* X = nullptr,
                              int px = 0);
// generalised least squares (gls.hip): the level-(M-1) multi-column leaf
// products of the reduce-order regions [q0, q1), and the whole call
hipError_t launch_gls_leaf(const mra_plan_s& H, const DevPlan& P, int64_t q0, int64_t q1, int R, hipStream_t st);
hipError_t launch_gls(const mra_plan_s& H, const double* y, const double* X, int p, const double* theta, double* beta,
                      double* out_ll, double* xtsix, double* grad, double* resid, hipStream_t st);

}  // namespace mra
