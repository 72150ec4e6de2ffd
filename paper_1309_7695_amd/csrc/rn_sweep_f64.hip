// rn_sweep_f64.hip -- the sweep kernels with every step in FP64 (the form whose
// trajectories match the FP64 reference bit for bit).
#include "rn_sweep_kernel.h"

namespace rn {

hipError_t launch_sweep_f64(const SweepParams& p, const LaunchCfg& cfg, hipStream_t stream) {
  return launch_sweep_prec<double>(p, cfg, stream);
}

hipError_t launch_persistent_f64(const BatchQueue& q, const LaunchCfg& cfg, hipStream_t stream,
                                 int64_t groups) {
  return launch_persistent_prec<double>(q, cfg, stream, groups);
}

}  // namespace rn
