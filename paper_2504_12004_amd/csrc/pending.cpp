// Entry points whose kernels are not in this build yet: they fail loudly.
#include "../../include/sbv.h"
#include <string>
sbv_status sbv_internal_fail(sbv_status st, const char* msg);
extern "C" {
sbv_status sbv_loglik_grad(const sbv_blocks*, int32_t, const double*, const int32_t*, int32_t, double*, double*) {
  return sbv_internal_fail(SBV_E_INVAL, "sbv_loglik_grad is not available in this build");
}
sbv_status sbv_loglik_grad_dev(const sbv_blocks*, int32_t, const double*, const int32_t*, int32_t, double*,
                               double*, void*) {
  return sbv_internal_fail(SBV_E_INVAL, "sbv_loglik_grad_dev is not available in this build");
}
}
