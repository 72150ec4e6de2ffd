// rn_plan.h -- internal: a validated sweep ready to launch, shared by rn_sweep
// and the batched launch.
#pragma once
#include <hip/hip_runtime.h>

#include "rn.h"
#include "rn_kernel.h"

namespace rn_internal {

struct SweepPlan {
  const rn_network* net = nullptr;
  bool empty = false;          // n_traj == 0: nothing to launch
  int32_t precision = RN_FP64;
  hipFunction_t fn = nullptr;  // network-compiled kernel, or null for the generic one
  int wg = 0;                  // workgroup size of the network-compiled kernel
  size_t lds = 0;              // its dynamic LDS bytes
  bool ssa_dep = false;        // it is the dependency-graph exact-SSA kernel
  bool wave = false;           // the one-wave-per-trajectory kernel (rn_wsweep.hip)
  int n_simd = 0;              // the device's SIMDs (4 per compute unit)
  rn::LaunchCfg cfg{};         // generic kernel configuration
  size_t lane_lds = 0;         // generic kernel LDS bytes per lane
  int max_segs = 0;            // rate register vectors of the generic kernel (0: rates in memory)
  int32_t n_species = 0, n_reactions = 0, nnz = 0;
  rn::SweepParams p{};
};

// Validate the arguments and choose the kernel.  wait_compile: compile the
// network's kernel now if needed; otherwise use it only when already compiled
// (starting its compilation in the background).  Returns RN_OK or RN_E_*.
int plan_sweep(const rn_network* net, const rn_sweep_args* a, SweepPlan& plan,
               bool wait_compile = true);
// Enqueue the sweep on `stream` (with the network's table copy if this is its
// first use).
hipError_t launch_plan(const SweepPlan& plan, hipStream_t stream);
// Copy the network's tables on the library stream now and wait for the copy
// (for launches recorded into a graph).
hipError_t stage_network_now(const rn_network* net);
// RN_OK for hipSuccess, else RN_E_DEVICE (recording the HIP code).
int device_status(hipError_t e);
// Start compiling the network's kernel in the background if it is not cached
// and a sweep of n_traj trajectories would use it (the launch shape follows
// n_traj as in plan_sweep).
void prefetch_kernel(const rn_network* net, int32_t precision, int64_t n_traj);

}  // namespace rn_internal
