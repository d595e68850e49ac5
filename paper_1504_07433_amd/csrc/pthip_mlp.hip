// pthip_mlp.hip -- learned surrogate of the Mandel-Agol functions.
#include "../../include/pthip.h"
#include "pthip_internal.h"

extern "C" {

static pt_status unsupported() { return PT_ERR_UNSUPPORTED; }

pt_status pt_mlp_datagen(const double*, int64_t, double*, void*) { return unsupported(); }
pt_status pt_mlp_forward(const pt_mlp*, const float*, int64_t, float*, float*, void*) { return unsupported(); }
pt_status pt_mlp_backward(const pt_mlp*, const float*, const float*, const float*, int64_t, pt_mlp*, void*) {
  return unsupported();
}
pt_status pt_mlp_adam_step(pt_mlp*, const pt_mlp*, pt_mlp*, pt_mlp*, int64_t, float, float, float, float, void*) {
  return unsupported();
}
pt_status pt_surrogate_set(const pt_mlp*, double, double, double, void*) { return unsupported(); }
pt_status pt_surrogate_eval(const double*, int64_t, double*, void*) { return unsupported(); }
}
