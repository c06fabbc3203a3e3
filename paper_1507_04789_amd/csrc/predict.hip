// Kriging pass of the M-RA (Prop. 2).
#include "cov.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace mra {

hipError_t launch_predict(const mra_plan_s& H, const double* theta, double* mean, double* var, hipStream_t st) {
  (void)H; (void)theta; (void)mean; (void)var; (void)st;
  return hipErrorNotSupported;
}

}  // namespace mra
