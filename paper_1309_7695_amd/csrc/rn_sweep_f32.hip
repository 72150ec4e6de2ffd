// rn_sweep_f32.hip -- the sweep kernels with FP32 propensities, SSA events,
// leap-condition bound and Poisson means (FP64 kept for time, the SSA-switch
// test, the critical race and the large-mean samplers).
#include "rn_sweep_kernel.h"

namespace rn {

hipError_t launch_sweep_f32(const SweepParams& p, const LaunchCfg& cfg, hipStream_t stream) {
  return launch_sweep_prec<float>(p, cfg, stream);
}

hipError_t launch_persistent_f32(const BatchQueue& q, const LaunchCfg& cfg, hipStream_t stream,
                                 int64_t groups) {
  return launch_persistent_prec<float>(q, cfg, stream, groups);
}

}  // namespace rn
