// Launch helper shared by the kernel files: a batch of independent tasks is
// one launch (grid.x = tasks, grid.y = parameter vectors), or, in the plain
// comparison form, one launch per task.  With profiling enabled every launch
// group is bracketed by HIP events on the call's stream.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "devplan.hpp"

struct mra_plan_s;

namespace mra {

// Task index of a workgroup.  Batched launches of tasks that share inputs
// (G consecutive task indices) place each group on one XCD: workgroups are
// dispatched to the 8 XCDs round-robin by block index, so block b runs on
// XCD b % 8; group g goes to XCD g % 8, and its G tasks take consecutive
// slots there, so they find the group's inputs in that XCD's L2.  Blocks
// past the last group return -1.
struct TaskMap {
  int64_t t0;     // first task (plain form: the single task of the launch)
  int64_t ntask;  // tasks in the launch (a multiple of G when G > 1)
  int32_t G;      // group size; 1 = identity mapping
};

__device__ __forceinline__ int64_t task_of(const TaskMap& m) {
  const int64_t b = blockIdx.x;
  if (m.G <= 1) return m.t0 + b;
  const int64_t xcd = b & 7, s = b >> 3;
  const int64_t g = (s / m.G) * 8 + xcd;
  if (g * m.G >= m.ntask) return -1;
  return m.t0 + g * m.G + (s % m.G);
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
  template <class K, class... A>
  void operator()(const char* name, int level, double flops, K kern, int64_t ntask, A... args) const {
    grouped(name, level, flops, 1, kern, ntask, args...);
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
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof && prof->enabled) {
      e0 = prof->next();
      e1 = prof->next();
      if (e0) (void)hipEventRecord(e0, st);
    }
    if (plain) {
      for (int64_t t = t_begin; t < t_end; ++t)
        hipLaunchKernelGGL(kern, dim3(1, nth), dim3(256), 0, st, P, args..., TaskMap{t, 1, 1});
    } else if (G <= 1) {
      hipLaunchKernelGGL(kern, dim3((unsigned)ntask, nth), dim3(256), 0, st, P, args..., TaskMap{t_begin, ntask, 1});
    } else {
      const int64_t ngroups = ntask / G;
      const int64_t nblk = (ngroups + 7) / 8 * 8 * G;
      hipLaunchKernelGGL(kern, dim3((unsigned)nblk, nth), dim3(256), 0, st, P, args..., TaskMap{t_begin, ntask, G});
    }
    if (e0 && e1) {
      (void)hipEventRecord(e1, st);
      prof->recs.push_back(ProfRecord{name, level, flops * nth, plain ? ntask : 1, e0, e1});
    }
  }
};

hipError_t launch_forward(const mra_plan_s& H, const double* y, const double* theta, int nth, double* out_loglik,
                          hipStream_t st);
hipError_t launch_forward_front(const mra_plan_s& H, const double* y, const double* theta, int nth, hipStream_t st,
                                hipStream_t side = nullptr, void* ev_fork = nullptr, void* ev_join = nullptr);
hipError_t launch_forward_back(const mra_plan_s& H, int nth, double* out_loglik, hipStream_t st);
hipError_t launch_grad_leafsolve(const mra_plan_s& H, int nth, hipStream_t st);
hipError_t launch_grad_post(const mra_plan_s& H, int nth, hipStream_t st);
hipError_t launch_grad_rest(const mra_plan_s& H, const double* theta, int nth, double* out_grad, hipStream_t st);

}  // namespace mra
