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
//
// Persistent form (rn_batch_persistent): every job runs the generic kernel
// body, and the jobs that share a launch shape (precision, trajectories per
// workgroup, rate registers) form one device work queue of (job, block) items,
// largest jobs first; one persistent kernel per shape takes items until its
// queue is empty, so workgroups move from job to job instead of each job's
// grid ending on its own tail.  The shapes' kernels are branches of one graph,
// after a node that zeroes the queue counters.  rn_batch_tune picks each job's
// shape and wave-scheduling threshold by timing short trials, per bucket of
// (species, reactions, stoichiometry entries), and keeps the choices for the
// process and, with RN_TUNE_CACHE set, in that file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "rn.h"
#include "rn_plan.h"

struct rn_batch {
  std::vector<rn_internal::SweepPlan> plans;
  std::vector<double> work;  // trajectory count as a load estimate
  int device = -1;
  bool persistent = false;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<hipStream_t> streams;  // [0] origin, then branches
  std::vector<hipEvent_t> events;
  void* dmem = nullptr;  // queues of the persistent form
};

namespace {

// A launch shape of the persistent form.
struct Shape {
  int wg = 64;        // trajectories per workgroup
  int segs = 0;       // rate register vectors (0: rates read from memory)
  float theta = 0.5f; // wave-scheduling threshold
};

// Tuned shapes by (precision, species/8, reactions/16, entries/32).
typedef std::tuple<int, int, int, int> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tuned;
bool g_tune_loaded = false;

TuneKey tune_key(const rn_internal::SweepPlan& pl) {
  return TuneKey(pl.precision, (pl.n_species + 7) / 8, (pl.n_reactions + 15) / 16,
                 (pl.nnz + 31) / 32);
}

const char* tune_file() {
  const char* f = std::getenv("RN_TUNE_CACHE");
  return f && f[0] ? f : nullptr;
}

// With g_tune_mu held: read the cache file once ("prec n m z wg segs theta" lines).
void load_tuned() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* f = tune_file();
  if (!f) return;
  FILE* fp = std::fopen(f, "r");
  if (!fp) return;
  int pr, n, m, z, wg, segs;
  float th;
  while (std::fscanf(fp, "%d %d %d %d %d %d %f", &pr, &n, &m, &z, &wg, &segs, &th) == 7)
    if ((wg == 64 || wg == 256) && segs >= 0 && segs <= 8 && th >= 0.0f && th <= 1.0f)
      g_tuned[TuneKey(pr, n, m, z)] = Shape{wg, segs, th};
  std::fclose(fp);
}

// With g_tune_mu held: write every tuned shape to the cache file.
void save_tuned() {
  const char* f = tune_file();
  if (!f) return;
  FILE* fp = std::fopen(f, "w");
  if (!fp) return;
  for (const auto& kv : g_tuned)
    std::fprintf(fp, "%d %d %d %d %d %d %.3f\n", std::get<0>(kv.first), std::get<1>(kv.first),
                 std::get<2>(kv.first), std::get<3>(kv.first), kv.second.wg, kv.second.segs,
                 kv.second.theta);
  std::fclose(fp);
}

// A job's shape: the tuned one for its bucket, else 64-lane workgroups (jobs
// share the chip, so smaller blocks balance better), its plan's rate
// registers and threshold.
Shape shape_of(const rn_internal::SweepPlan& pl) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  load_tuned();
  auto it = g_tuned.find(tune_key(pl));
  if (it != g_tuned.end() && (it->second.segs == 0 || it->second.segs == pl.max_segs))
    return it->second;
  return Shape{64, pl.max_segs, pl.p.theta};
}

hipError_t launch_persistent(int precision, const rn::BatchQueue& q, const rn::LaunchCfg& cfg,
                             hipStream_t st, int64_t groups) {
  return precision == RN_FP32 ? rn::launch_persistent_f32(q, cfg, st, groups)
                              : rn::launch_persistent_f64(q, cfg, st, groups);
}

int cu_count(int dev) {
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
  return n > 0 ? n : 1;
}

// Parallel branches of the graph: RN_BATCH_BRANCHES (1..64), default 8.  Kernels
// on more branches than the process has hardware queues (GPU_MAX_HW_QUEUES)
// share queues and run in turn.
int branches() {
  const char* e = std::getenv("RN_BATCH_BRANCHES");
  const int v = e ? std::atoi(e) : 8;
  return v >= 1 && v <= 64 ? v : 8;
}

void release(rn_batch* b) {
  if (b->dmem) (void)hipFree(b->dmem);
  b->dmem = nullptr;
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

// LDS class of a job: the bit width of its bytes per lane.  A persistent
// workgroup holds the largest LDS of its group, so jobs of very different
// footprints go to different groups.
int lds_class(size_t lane_lds) {
  int c = 0;
  while (lane_lds > 0) {
    lane_lds >>= 1;
    ++c;
  }
  return c;
}

// One persistent group: jobs of one shape, precision and LDS class.
struct Group {
  int precision;
  int lclass;
  Shape shape;
  std::vector<size_t> jobs;
  size_t lds = 0;
  std::vector<int32_t> items;  // (job, block) pairs
};

// The persistent form: queues in one device block (job parameters, items,
// counters), then the graph: zero the counters and the jobs' fused
// statistics, fork one persistent kernel per group, join, finish statistics.
hipError_t capture_persistent(rn_batch* b) {
  const int n_cu = cu_count(b->device);
  std::vector<Group> groups;
  std::vector<rn::SweepParams> params(b->plans.size());
  std::vector<size_t> wave_jobs;  // jobs on the one-wave-per-trajectory kernel
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const rn_internal::SweepPlan& pl = b->plans[i];
    params[i] = pl.p;
    if (pl.wave) {
      wave_jobs.push_back(i);
      continue;
    }
    const Shape sh = shape_of(pl);
    params[i].theta = sh.theta;
    params[i].phase_cycles = nullptr;
    const int lc = lds_class(pl.lane_lds);
    size_t g = 0;
    while (g < groups.size() &&
           !(groups[g].precision == pl.precision && groups[g].lclass == lc &&
             groups[g].shape.wg == sh.wg && groups[g].shape.segs == sh.segs))
      ++g;
    if (g == groups.size()) groups.push_back(Group{pl.precision, lc, sh, {}, 0, {}});
    groups[g].jobs.push_back(i);
    groups[g].lds = std::max(groups[g].lds, pl.lane_lds * (size_t)sh.wg);
  }
  // items: the jobs of a group by decreasing work (trajectories x reactions),
  // each job's blocks in order
  for (Group& gr : groups) {
    std::stable_sort(gr.jobs.begin(), gr.jobs.end(), [&](size_t x, size_t y) {
      return b->work[x] * b->plans[x].n_reactions > b->work[y] * b->plans[y].n_reactions;
    });
    for (size_t i : gr.jobs) {
      const int64_t blocks = (b->plans[i].p.n_traj + gr.shape.wg - 1) / gr.shape.wg;
      for (int64_t k = 0; k < blocks; ++k) {
        gr.items.push_back((int32_t)i);
        gr.items.push_back((int32_t)k);
      }
    }
  }
  const size_t pbytes = (params.size() * sizeof(rn::SweepParams) + 255) / 256 * 256;
  size_t ibytes = 0;
  for (const Group& gr : groups) ibytes += (gr.items.size() * sizeof(int32_t) + 255) / 256 * 256;
  const size_t cbytes = groups.size() * sizeof(uint32_t);
  hipError_t e = hipMalloc(&b->dmem, pbytes + ibytes + cbytes);
  if (e != hipSuccess) return e;
  char* base = (char*)b->dmem;
  e = hipMemcpy(base, params.data(), params.size() * sizeof(rn::SweepParams),
                hipMemcpyHostToDevice);
  std::vector<rn::BatchQueue> queues(groups.size());
  size_t off = pbytes;
  uint32_t* counters = (uint32_t*)(base + pbytes + ibytes);
  for (size_t g = 0; g < groups.size() && e == hipSuccess; ++g) {
    e = hipMemcpy(base + off, groups[g].items.data(), groups[g].items.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice);
    queues[g] = rn::BatchQueue{(const rn::SweepParams*)base, (const int32_t*)(base + off),
                               (int32_t)(groups[g].items.size() / 2), counters + g};
    off += (groups[g].items.size() * sizeof(int32_t) + 255) / 256 * 256;
  }
  if (e != hipSuccess) return e;

  // the wave jobs on their own branches (at most four), largest first, each to
  // the branch with the fewest trajectories
  const int nw = (int)std::min<size_t>(wave_jobs.size(), 4);
  std::stable_sort(wave_jobs.begin(), wave_jobs.end(), [&](size_t x, size_t y) {
    return b->work[x] * b->plans[x].n_reactions > b->work[y] * b->plans[y].n_reactions;
  });
  const int nb = (int)groups.size();
  for (int k = 0; k < nb + nw + 1; ++k) {
    hipStream_t st = nullptr;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return e;
    b->streams.push_back(st);
    hipEvent_t ev = nullptr;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    b->events.push_back(ev);
  }
  hipStream_t origin = b->streams[0];
  if ((e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipError_t err = rn::launch_fill_u32(counters, (int64_t)groups.size(), 0u, origin);
  // (a wave job's launch_plan zeroes and finishes its own statistics)
  for (size_t i = 0; i < params.size() && err == hipSuccess; ++i)
    if (!b->plans[i].wave && (params[i].sum_x || params[i].hist))
      err = rn::launch_stats_zero(params[i], origin);
  if (err == hipSuccess) err = hipEventRecord(b->events[0], origin);
  std::vector<double> wload(nw, 0.0);
  for (size_t i : wave_jobs) {
    if (err != hipSuccess) break;
    int k = 0;
    for (int q = 1; q < nw; ++q)
      if (wload[q] < wload[k]) k = q;
    hipStream_t st = b->streams[nb + 1 + k];
    if (wload[k] == 0.0) err = hipStreamWaitEvent(st, b->events[0], 0);
    wload[k] += b->work[i];
    if (err == hipSuccess) err = rn_internal::launch_plan(b->plans[i], st);
  }
  for (int k = 0; k < nw && err == hipSuccess; ++k) {
    err = hipEventRecord(b->events[nb + 1 + k], b->streams[nb + 1 + k]);
    if (err == hipSuccess) err = hipStreamWaitEvent(origin, b->events[nb + 1 + k], 0);
  }
  for (int g = 0; g < nb && err == hipSuccess; ++g) {
    hipStream_t st = b->streams[g + 1];
    err = hipStreamWaitEvent(st, b->events[0], 0);
    rn::LaunchCfg cfg{groups[g].shape.wg, groups[g].shape.segs, groups[g].lds};
    // one workgroup per SIMD's worth of lanes on every compute unit
    const int64_t grid = std::min<int64_t>((int64_t)queues[g].n_items,
                                           (int64_t)n_cu * (256 / groups[g].shape.wg));
    if (err == hipSuccess) err = launch_persistent(groups[g].precision, queues[g], cfg, st, grid);
    if (err == hipSuccess) err = hipEventRecord(b->events[g + 1], st);
    if (err == hipSuccess) err = hipStreamWaitEvent(origin, b->events[g + 1], 0);
  }
  for (size_t i = 0; i < params.size() && err == hipSuccess; ++i)
    if (!b->plans[i].wave && params[i].sum_x) err = rn::launch_stats_finish(params[i], origin);
  hipGraph_t gph = nullptr;
  e = hipStreamEndCapture(origin, &gph);
  if (err != hipSuccess) {
    if (gph) (void)hipGraphDestroy(gph);
    return err;
  }
  if (e != hipSuccess) return e;
  b->graph = gph;
  return hipGraphInstantiate(&b->exec, gph, nullptr, nullptr, 0);
}

// Steps per trajectory in a tuning trial: every candidate shape runs the same
// bounded work whatever the job's horizon.
constexpr uint64_t kTrialSteps = 400;

// Time one persistent launch of the trajectories [0, n) of plan `pl`, each
// stopped after kTrialSteps steps, in shape `sh` (without fused statistics);
// milliseconds of the last of `reps` runs.
hipError_t trial(const rn_internal::SweepPlan& pl, const Shape& sh, int64_t n, int reps,
                 hipStream_t st, int n_cu, float* ms) {
  rn::SweepParams p = pl.p;
  p.n_traj = n;
  p.max_steps = std::min<uint64_t>(p.max_steps, kTrialSteps);
  p.theta = sh.theta;
  p.phase_cycles = nullptr;
  p.sum_x = nullptr;
  p.sum_x2 = nullptr;
  p.hist = nullptr;
  const int64_t blocks = (n + sh.wg - 1) / sh.wg;
  std::vector<int32_t> items;
  for (int64_t k = 0; k < blocks; ++k) {
    items.push_back(0);
    items.push_back((int32_t)k);
  }
  const size_t pbytes = (sizeof(p) + 255) / 256 * 256;
  const size_t ibytes = (items.size() * sizeof(int32_t) + 255) / 256 * 256;
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, pbytes + ibytes + 256);
  if (e != hipSuccess) return e;
  char* base = (char*)mem;
  uint32_t* counter = (uint32_t*)(base + pbytes + ibytes);
  e = hipMemcpy(base, &p, sizeof(p), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + pbytes, items.data(), items.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice);
  const rn::BatchQueue q{(const rn::SweepParams*)base, (const int32_t*)(base + pbytes),
                         (int32_t)blocks, counter};
  const rn::LaunchCfg cfg{sh.wg, sh.segs, pl.lane_lds * (size_t)sh.wg};
  const int64_t grid = std::min<int64_t>(blocks, (int64_t)n_cu * (256 / sh.wg));
  hipEvent_t a = nullptr, z = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&z);
  float best = 0.0f;
  for (int rep = 0; rep < reps && e == hipSuccess; ++rep) {
    e = rn::launch_fill_u32(counter, 1, 0u, st);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch_persistent(pl.precision, q, cfg, st, grid);
    if (e == hipSuccess) e = hipEventRecord(z, st);
    if (e == hipSuccess) e = hipEventSynchronize(z);
    if (e == hipSuccess) e = hipEventElapsedTime(&best, a, z);
  }
  if (a) (void)hipEventDestroy(a);
  if (z) (void)hipEventDestroy(z);
  (void)hipFree(mem);
  *ms = best;
  return e;
}

}  // namespace

extern "C" {

int rn_batch_persistent(rn_batch* b, int32_t on) {
  if (!b || b->exec) return RN_E_INVALID_ARG;
  b->persistent = on != 0;
  return RN_OK;
}

int rn_batch_tune(rn_batch* b, void* hip_stream) {
  if (!b || b->exec) return RN_E_INVALID_ARG;
  if (b->plans.empty()) return RN_OK;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rn_internal::device_status(e);
  if (dev != b->device) return RN_E_INVALID_ARG;
  const int n_cu = cu_count(dev);
  hipStream_t st = (hipStream_t)hip_stream;
  // the largest job of every bucket not tuned yet
  std::map<TuneKey, size_t> todo;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_tuned();
    for (size_t i = 0; i < b->plans.size(); ++i) {
      if (b->plans[i].wave) continue;  // not a work-queue job
      const TuneKey k = tune_key(b->plans[i]);
      if (g_tuned.count(k)) continue;
      auto it = todo.find(k);
      if (it == todo.end() || b->work[i] > b->work[it->second]) todo[k] = i;
    }
  }
  // RN_TUNE_LOG=1: one line per bucket on stderr as it is tuned
  const char* lg = std::getenv("RN_TUNE_LOG");
  const bool log = lg && lg[0] == '1';
  size_t done = 0;
  for (const auto& kv : todo) {
    const rn_internal::SweepPlan& pl = b->plans[kv.second];
    // a trial: up to one wave per SIMD of trajectories; the bucket's first
    // candidate runs twice (loading its code), the others once
    const int64_t n = std::min<int64_t>(pl.p.n_traj, (int64_t)n_cu * 256);
    int reps = 2;
    Shape best{64, pl.max_segs, pl.p.theta};
    float best_ms = 0.0f;
    bool have = false;
    for (int wg : {64, 256}) {
      for (int segs : {pl.max_segs, 0}) {
        for (float th : {0.35f, 0.5f, 0.65f}) {
          // the persistent kernel's own item word shares the 160 KiB
          if (pl.lane_lds * (size_t)wg + 64 > 160 * 1024) continue;
          float ms = 0.0f;
          e = trial(pl, Shape{wg, segs, th}, n, reps, st, n_cu, &ms);
          reps = 1;
          if (e != hipSuccess) return rn_internal::device_status(e);
          if (!have || ms < best_ms) {
            best = Shape{wg, segs, th};
            best_ms = ms;
            have = true;
          }
        }
        if (pl.max_segs == 0) break;  // only one rate placement
      }
    }
    if (log)
      std::fprintf(stderr, "rn_batch_tune: bucket %zu/%zu (N %d, M %d): wg %d, rate vectors %d, "
                   "theta %.2f, %.2f ms\n", ++done, todo.size(), pl.n_species, pl.n_reactions,
                   best.wg, best.segs, best.theta, best_ms);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[kv.first] = best;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (!todo.empty()) save_tuned();
  return RN_OK;
}

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
    e = b->persistent ? capture_persistent(b) : capture(b);
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
