// Placeholder until the U-Net kernels land: the learned preconditioner
// reports itself unavailable, so LEARNED contexts solve with MIC(0).
#include "net.h"

namespace fs {

size_t net_workspace_bytes(int) { return 256; }
int net_init(sim_ctx*) { return SIM_OK; }
void net_destroy(sim_ctx*) {}
bool net_ready(const sim_ctx*) { return false; }
int net_apply(sim_ctx* c, const float*, float*, const int*) {
  c->err = "learned preconditioner not available";
  return SIM_ERR_STATE;
}

}  // namespace fs

extern "C" {
int sim_net_param_count(int64_t* count) {
  if (!count) return SIM_ERR_INVALID_ARG;
  *count = 353808;
  return SIM_OK;
}
int sim_net_set_weights(sim_ctx* c, const float*, int64_t) {
  if (!c) return SIM_ERR_INVALID_ARG;
  c->err = "learned preconditioner not available";
  return SIM_ERR_STATE;
}
int sim_net_forward(sim_ctx* c, const float*, float*) {
  if (!c) return SIM_ERR_INVALID_ARG;
  c->err = "learned preconditioner not available";
  return SIM_ERR_STATE;
}
int sim_net_train_step(sim_ctx* c, const float*, const float*, int32_t, float*, float*, int32_t,
                       float, double*) {
  if (!c) return SIM_ERR_INVALID_ARG;
  c->err = "learned preconditioner not available";
  return SIM_ERR_STATE;
}
}
