// Learned-dynamics extension (placeholder until the MLP kernels land).
#include "mppi_runtime.h"

namespace mppi {
uint64_t extra_workspace_bytes(const mppi_config *) { return 0; }
int init_extra(mppi_ctx *, const mppi_config *cfg) {
  if (cfg->system == MPPI_SYS_QUADROTOR_MLP) return fail(MPPI_EINVAL, "learned dynamics not available in this build");
  return MPPI_OK;
}
void destroy_extra(mppi_ctx *) {}
int launch_mlp_rollout(mppi_ctx *, const IterArgs &, hipStream_t) { return fail(MPPI_EINVAL, "learned dynamics not available"); }
}  // namespace mppi
