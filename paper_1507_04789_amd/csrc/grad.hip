// Reverse pass (gradient) of the M-RA log-likelihood.
#include "cov.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace mra {

hipError_t launch_grad(const mra_plan_s& H, const double* theta, int nth, double* out_grad, hipStream_t st) {
  (void)H; (void)theta; (void)nth; (void)out_grad; (void)st;
  return hipErrorNotSupported;
}

}  // namespace mra
