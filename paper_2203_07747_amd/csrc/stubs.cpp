// Entry points of the header whose kernels are not built yet: they validate
// nothing and report RTN_ENOTSUP so that callers fail loudly.
#include <hip/hip_runtime.h>

#include "../../include/rtn.h"

extern "C" {

rtn_status rtn_mlp_forward(rtn_model*, int32_t, int32_t, const float*, float*, void*) { return RTN_ENOTSUP; }
rtn_status rtn_mlp_backward(rtn_model*, int32_t, const float*, float*, void*) { return RTN_ENOTSUP; }
rtn_status rtn_model_zero_grad(rtn_model*, void*) { return RTN_ENOTSUP; }
rtn_status rtn_model_get_grad(rtn_model*, float*) { return RTN_ENOTSUP; }
rtn_status rtn_adam_step(rtn_model*, float, float, float, float, void*) { return RTN_ENOTSUP; }
rtn_status rtn_train_step(rtn_model*, int32_t, int32_t, const float*, const float*, float, float, float, float, float*,
                          void*) {
  return RTN_ENOTSUP;
}
rtn_status rtn_model_get_adam(rtn_model*, float*, float*, int64_t*) { return RTN_ENOTSUP; }
rtn_status rtn_model_set_adam(rtn_model*, const float*, const float*, int64_t) { return RTN_ENOTSUP; }
}
