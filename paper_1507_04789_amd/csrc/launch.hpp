// Launch helper shared by the kernel files: a batch of independent tasks is
// one launch (grid.x = tasks, grid.y = parameter vectors), or, in the plain
// comparison form, one launch per task.
#pragma once
#include <hip/hip_runtime.h>

#include "devplan.hpp"

struct mra_plan_s;

namespace mra {

struct Runner {
  const DevPlan& P;
  int nth;
  hipStream_t st;
  bool plain;
  template <class K, class... A>
  void operator()(K kern, int64_t ntask, A... args) const {
    if (ntask <= 0) return;
    if (plain) {
      for (int64_t t = 0; t < ntask; ++t)
        hipLaunchKernelGGL(kern, dim3(1, nth), dim3(256), 0, st, P, args..., t);
    } else {
      hipLaunchKernelGGL(kern, dim3((unsigned)ntask, nth), dim3(256), 0, st, P, args..., (int64_t)0);
    }
  }
};

hipError_t launch_forward(const mra_plan_s& H, const double* y, const double* theta, int nth, double* out_loglik,
                          hipStream_t st);

}  // namespace mra
