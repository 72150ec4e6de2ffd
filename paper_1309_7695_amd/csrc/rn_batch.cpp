// rn_batch.cpp -- many sweep jobs (networks of any size, any trajectory count)
// launched together through one HIP graph.
//
// The jobs are independent (paper, Aims and motivation section: sweeps repeat
// many simulations), so the graph runs them as parallel branches: the first
// launch forks from an internal origin stream onto a small pool of branch
// streams, enqueues each job's kernel on one branch (largest jobs first, each
// to the least-loaded branch), joins, and captures the whole pattern; every
// later launch replays it with a single hipGraphLaunch on the caller's stream.
// Small jobs then fill the compute units that large ones leave idle, and the
// host cost of a batch is one launch.  The graph holds kernel nodes only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <new>
#include <vector>

#include "rn.h"
#include "rn_plan.h"

struct rn_batch {
  std::vector<rn_internal::SweepPlan> plans;
  std::vector<double> work;  // trajectory count as a load estimate
  int device = -1;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<hipStream_t> streams;  // [0] origin, then branches
  std::vector<hipEvent_t> events;
};

namespace {

// Parallel branches of the graph: RN_BATCH_BRANCHES (1..64), default 8.  Kernels
// on more branches than the process has hardware queues (GPU_MAX_HW_QUEUES)
// share queues and run in turn.
int branches() {
  const char* e = std::getenv("RN_BATCH_BRANCHES");
  const int v = e ? std::atoi(e) : 8;
  return v >= 1 && v <= 64 ? v : 8;
}

void release(rn_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  b->exec = nullptr;
  b->graph = nullptr;
  b->events.clear();
  b->streams.clear();
}

// Record the fork, the job launches and the join on the origin stream.
hipError_t capture(rn_batch* b) {
  const int nb = (int)std::min<size_t>((size_t)branches(), std::max<size_t>(1, b->plans.size()));
  hipError_t e;
  for (int k = 0; k < nb + 1; ++k) {
    hipStream_t s = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return e;
    b->streams.push_back(s);
  }
  for (int k = 0; k < nb + 1; ++k) {
    hipEvent_t ev = nullptr;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    b->events.push_back(ev);
  }
  hipStream_t origin = b->streams[0];
  if ((e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipError_t err = hipEventRecord(b->events[0], origin);
  for (int k = 1; k <= nb && err == hipSuccess; ++k)
    err = hipStreamWaitEvent(b->streams[k], b->events[0], 0);
  // largest jobs first, each onto the least-loaded branch
  std::vector<size_t> order(b->plans.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return b->work[x] > b->work[y]; });
  std::vector<double> load(nb + 1, 0.0);
  for (size_t i : order) {
    if (err != hipSuccess) break;
    int k = 1;
    for (int q = 2; q <= nb; ++q)
      if (load[q] < load[k]) k = q;
    load[k] += b->work[i];
    err = rn_internal::launch_plan(b->plans[i], b->streams[k]);
  }
  for (int k = 1; k <= nb && err == hipSuccess; ++k) {
    err = hipEventRecord(b->events[k], b->streams[k]);
    if (err == hipSuccess) err = hipStreamWaitEvent(origin, b->events[k], 0);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(origin, &g);
  if (err != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return err;
  }
  if (e != hipSuccess) return e;
  b->graph = g;
  return hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
}

}  // namespace

extern "C" {

int rn_batch_create(rn_batch** out) {
  if (!out) return RN_E_INVALID_ARG;
  rn_batch* b = new (std::nothrow) rn_batch;
  if (!b) return RN_E_NOMEM;
  *out = b;
  return RN_OK;
}

int rn_batch_add(rn_batch* b, const rn_network* net, const rn_sweep_args* args) {
  if (!b || !net || !args) return RN_E_INVALID_ARG;
  if (b->exec) return RN_E_INVALID_ARG;  // the graph is fixed after the first launch
  rn_internal::SweepPlan plan;
  const int rc = rn_internal::plan_sweep(net, args, plan);
  if (rc != RN_OK) return rc;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RN_E_DEVICE;
  if (b->device >= 0 && dev != b->device) return RN_E_INVALID_ARG;
  b->device = dev;
  if (plan.empty) return RN_OK;
  // the graph's kernels then read tables that are already in place
  const hipError_t se = rn_internal::stage_network_now(net);
  if (se != hipSuccess) return rn_internal::device_status(se);
  try {
    b->plans.push_back(plan);
    b->work.push_back((double)args->n_traj);
  } catch (const std::bad_alloc&) {
    return RN_E_NOMEM;
  }
  return RN_OK;
}

int rn_batch_size(const rn_batch* b) { return b ? (int)b->plans.size() : RN_E_INVALID_ARG; }

int rn_batch_launch(rn_batch* b, void* hip_stream) {
  if (!b) return RN_E_INVALID_ARG;
  if (b->plans.empty()) return RN_OK;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rn_internal::device_status(e);
  if (dev != b->device) return RN_E_INVALID_ARG;
  if (!b->exec) {
    e = capture(b);
    if (e != hipSuccess) {
      release(b);
      return rn_internal::device_status(e);
    }
  }
  return rn_internal::device_status(hipGraphLaunch(b->exec, (hipStream_t)hip_stream));
}

void rn_batch_free(rn_batch* b) {
  if (!b) return;
  release(b);
  delete b;
}

}  // extern "C"
