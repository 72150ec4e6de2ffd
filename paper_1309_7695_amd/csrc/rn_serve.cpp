// rn_serve.cpp -- a sweep-job server: continuous admission of jobs of
// different networks and sizes into a fixed HBM budget.
//
// The device memory is one arena allocated at creation (the budget); every job
// takes one block of it (first fit, 256-byte aligned) for its inputs, samples
// and stats from admission on, so serving never calls hipMalloc.  Jobs are
// admitted strictly in arrival order whenever a block and a stream slot are
// free; each runs on one of a few streams, so jobs admitted while others run
// overlap on the device.  Progress happens inside the calls (submit, poll,
// fetch): there is no server thread.
//
// Host traffic stays on the job's own stream: when the pinned staging arena
// has room for the whole job, its inputs are copied from there before the
// kernel and its results back into it right after, so the device block is
// free again as soon as the job completes and fetching is a host memcpy.  A
// stream serves one job after another, and a copy queued on a stream that is
// already running a later job would wait for that kernel.
//
// A job never waits for its network's kernel to compile: the compilation
// starts in the background when the job is submitted, and the job runs the
// compiled kernel if it is ready by admission, else the generic kernel
// (identical results).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "rn.h"
#include "rn_plan.h"

namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, cap) with coalescing of freed blocks.
class Arena {
 public:
  void init(size_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, o = it->first;
      free_.erase(it);
      if (rest) free_[o + n] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }

 private:
  std::map<size_t, size_t> free_;
};

enum JobState { kQueued, kRunning, kDone };

struct Job {
  int64_t id = 0;
  const rn_network* net = nullptr;
  int64_t T = 0;
  int32_t S = 0, N = 0, M = 0, x0_per_traj = 0;
  std::vector<double> rates, times;  // host copies until completion (when not pinned)
  std::vector<int32_t> x0;
  bool pinned = false;               // inputs staged in the pinned arena instead
  bool pin_out = false;              // ... and results too (the block has the device layout)
  size_t pin_off = 0, pin_bytes = 0;
  bool dev_held = false;             // holds its device block
  rn_sweep_args params{};
  size_t bytes = 0, off = 0;
  size_t o_rates = 0, o_x0 = 0, o_times = 0, o_out = 0, o_stats = 0;  // within the block
  int stream = -1;
  hipEvent_t done = nullptr;
  JobState state = kQueued;
  bool reported = false;
  int rc = RN_OK;
};

}  // namespace

struct rn_server {
  int device = -1;
  char* base = nullptr;
  size_t cap = 0;
  Arena arena;
  // Pinned host staging for job inputs: copies from it are asynchronous, so
  // admitting a job never blocks behind kernels already running.
  char* pin = nullptr;
  size_t pin_cap = 0;
  Arena pin_arena;
  std::vector<hipStream_t> streams;
  std::vector<int> busy;  // running jobs per stream
  hipStream_t copy = nullptr;  // results of jobs without pinned results (never behind a job)
  int running = 0;
  int64_t next_id = 1;
  size_t in_use = 0;
  std::deque<Job*> queue;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  std::mutex mu;
};

namespace {

// Copy a job's inputs to its block and launch its sweep on stream k.
int start(rn_server* s, Job* j, int k) {
  char* blk = s->base + j->off;
  hipStream_t st = s->streams[k];
  hipError_t e;
  if (j->pinned) {  // inputs are laid out in the pinned block as in the device block
    e = hipMemcpyAsync(blk, s->pin + j->pin_off, j->pin_bytes, hipMemcpyHostToDevice, st);
  } else {
    e = hipMemcpyAsync(blk + j->o_rates, j->rates.data(), j->rates.size() * sizeof(double),
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(blk + j->o_x0, j->x0.data(), j->x0.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(blk + j->o_times, j->times.data(), j->times.size() * sizeof(double),
                         hipMemcpyHostToDevice, st);
  }
  if (e != hipSuccess) return rn_internal::device_status(e);
  rn_sweep_args a = j->params;
  a.n_traj = j->T;
  a.traj_offset = 0;
  a.rates = (const double*)(blk + j->o_rates);
  a.rates_ld = j->T;
  a.x0 = (const int32_t*)(blk + j->o_x0);
  a.x0_ld = j->x0_per_traj ? j->T : 0;
  a.times = (const double*)(blk + j->o_times);
  a.n_times = j->S;
  a.out = (int32_t*)(blk + j->o_out);
  a.out_ld = j->T;
  a.stats = (uint64_t*)(blk + j->o_stats);
  rn_internal::SweepPlan plan;
  int rc = rn_internal::plan_sweep(j->net, &a, plan, /*wait_compile=*/false);
  if (rc != RN_OK) return rc;
  e = rn_internal::launch_plan(plan, st);
  if (e == hipSuccess && j->pin_out)
    e = hipMemcpyAsync(s->pin + j->pin_off + j->o_out, blk + j->o_out,
                       (size_t)j->S * j->N * j->T * sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && j->pin_out)
    e = hipMemcpyAsync(s->pin + j->pin_off + j->o_stats, blk + j->o_stats,
                       (size_t)j->T * 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(j->done, st);
  if (e != hipSuccess) return rn_internal::device_status(e);
  // the asynchronous copies read the job's host vectors, which are kept until
  // the job's event completes (progress releases them then)
  return RN_OK;
}

void release_device(rn_server* s, Job* j) {
  if (!j->dev_held) return;
  s->arena.release(j->off, j->bytes);
  s->in_use -= j->bytes;
  j->dev_held = false;
}

void release_pinned(rn_server* s, Job* j) {
  if (!j->pinned) return;
  s->pin_arena.release(j->pin_off, j->pin_bytes);
  j->pinned = false;
  j->pin_out = false;
}

// Retire finished jobs and admit queued ones in arrival order.
void progress(rn_server* s) {
  for (auto& kv : s->jobs) {
    Job* j = kv.second.get();
    if (j->state != kRunning) continue;
    const hipError_t q = hipEventQuery(j->done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) j->rc = rn_internal::device_status(q);
    j->state = kDone;
    s->busy[j->stream]--;
    s->running--;
    j->rates = {};
    j->x0 = {};
    j->times = {};
    if (j->pin_out && j->rc == RN_OK)
      release_device(s, j);  // the results are in the pinned block
    else
      release_pinned(s, j);  // inputs only (or nothing to keep)
  }
  while (!s->queue.empty() && s->running < (int)s->streams.size()) {
    Job* j = s->queue.front();
    size_t off = 0;
    if (!s->arena.alloc(j->bytes, &off)) break;  // wait for memory, in order
    s->queue.pop_front();
    j->off = off;
    j->dev_held = true;
    s->in_use += j->bytes;
    int k = 0;
    for (int q = 1; q < (int)s->busy.size(); ++q)
      if (s->busy[q] < s->busy[k]) k = q;
    j->stream = k;
    s->busy[k]++;
    s->running++;
    j->state = kRunning;
    j->rc = start(s, j, k);
    if (j->rc != RN_OK) {  // nothing was launched after the failure point
      (void)hipStreamSynchronize(s->streams[k]);
      j->state = kDone;
      s->busy[k]--;
      s->running--;
    }
  }
}

}  // namespace

extern "C" {

int rn_server_create(int64_t hbm_budget_bytes, int32_t max_running, rn_server** out) {
  if (!out || hbm_budget_bytes <= 0 || max_running < 1 || max_running > 64)
    return RN_E_INVALID_ARG;
  rn_server* s = new (std::nothrow) rn_server;
  if (!s) return RN_E_NOMEM;
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipMalloc((void**)&s->base, (size_t)hbm_budget_bytes);
  if (e != hipSuccess) {
    delete s;
    return e == hipErrorOutOfMemory ? RN_E_NOMEM : rn_internal::device_status(e);
  }
  s->cap = (size_t)hbm_budget_bytes / kAlign * kAlign;
  s->arena.init(s->cap);
  s->pin_cap = std::min<size_t>(s->cap / 4, (size_t)4 << 30) / kAlign * kAlign;
  if (s->pin_cap && hipHostMalloc((void**)&s->pin, s->pin_cap, hipHostMallocDefault) != hipSuccess) {
    s->pin = nullptr;  // no pinned staging: inputs are copied from pageable memory
    s->pin_cap = 0;
  }
  s->pin_arena.init(s->pin_cap);
  for (int k = 0; k < max_running; ++k) {
    hipStream_t st = nullptr;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) break;
    s->streams.push_back(st);
    s->busy.push_back(0);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
  if (e != hipSuccess) {
    rn_server_free(s);
    return rn_internal::device_status(e);
  }
  *out = s;
  return RN_OK;
}

int rn_server_submit(rn_server* s, const rn_serve_job* job, int64_t* job_id) {
  if (!s || !job || !job_id || !job->net || job->n_traj < 1 || job->n_times < 1 ||
      !job->rates || !job->x0 || !job->times)
    return RN_E_INVALID_ARG;
  const int32_t N = rn_network_species(job->net), M = rn_network_reactions(job->net);
  if (N < 1 || M < 1) return RN_E_INVALID_ARG;
  std::lock_guard<std::mutex> lock(s->mu);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->device) return RN_E_INVALID_ARG;
  std::unique_ptr<Job> j;
  try {
    j.reset(new Job);
    j->net = job->net;
    j->T = job->n_traj;
    j->S = job->n_times;
    j->N = N;
    j->M = M;
    j->x0_per_traj = job->x0_per_traj ? 1 : 0;
    j->rates.assign(job->rates, job->rates + (size_t)M * job->n_traj);
    j->x0.assign(job->x0, job->x0 + (size_t)N * (j->x0_per_traj ? job->n_traj : 1));
    j->times.assign(job->times, job->times + job->n_times);
  } catch (const std::bad_alloc&) {
    return RN_E_NOMEM;
  }
  j->params = job->params;
  // the server writes the sample array; fused statistics are not served
  j->params.phase_cycles = nullptr;
  j->params.sum_x = nullptr;
  j->params.sum_x2 = nullptr;
  j->params.hist = nullptr;
  j->params.hist_lo = nullptr;
  j->params.hist_width = nullptr;
  j->params.hist_bins = 0;
  j->params.out_layout = RN_OUT_SAMPLE_MAJOR;
  // validate the method options now (sizes and pointers are the server's)
  {
    rn_sweep_args a = j->params;
    a.n_traj = 0;
    a.n_times = job->n_times;
    rn_internal::SweepPlan probe;
    const int rc = rn_internal::plan_sweep(job->net, &a, probe, false);
    if (rc != RN_OK) return rc;
  }
  size_t o = 0;
  j->o_rates = o;
  o += round_up(j->rates.size() * sizeof(double));
  j->o_x0 = o;
  o += round_up(j->x0.size() * sizeof(int32_t));
  j->o_times = o;
  o += round_up(j->times.size() * sizeof(double));
  j->o_out = o;
  o += round_up((size_t)j->S * N * j->T * sizeof(int32_t));
  j->o_stats = o;
  o += round_up((size_t)j->T * 4 * sizeof(uint64_t));
  j->bytes = o;
  if (j->bytes > s->cap) return RN_E_NOMEM;
  // Stage the job in pinned memory when there is room, with the layout of the
  // device block: the whole job (inputs and results), else the inputs only.
  const size_t in_bytes = j->o_out;
  size_t po = 0;
  if (s->pin && s->pin_arena.alloc(j->bytes, &po)) {
    j->pin_out = true;
    j->pin_bytes = j->bytes;
  } else if (s->pin && s->pin_arena.alloc(in_bytes, &po)) {
    j->pin_bytes = in_bytes;
  }
  if (j->pin_bytes) {
    char* b = s->pin + po;
    std::memcpy(b + j->o_rates, j->rates.data(), j->rates.size() * sizeof(double));
    std::memcpy(b + j->o_x0, j->x0.data(), j->x0.size() * sizeof(int32_t));
    std::memcpy(b + j->o_times, j->times.data(), j->times.size() * sizeof(double));
    j->pinned = true;
    j->pin_off = po;
    j->rates = {};
    j->x0 = {};
    j->times = {};
  }
  if (hipEventCreateWithFlags(&j->done, hipEventDisableTiming) != hipSuccess) {
    release_pinned(s, j.get());
    return RN_E_DEVICE;
  }
  rn_internal::prefetch_kernel(job->net, job->params.precision, job->n_traj);
  j->id = s->next_id++;
  *job_id = j->id;
  Job* raw = j.get();
  try {
    s->jobs.emplace(raw->id, std::move(j));
    s->queue.push_back(raw);
  } catch (const std::bad_alloc&) {
    return RN_E_NOMEM;
  }
  progress(s);
  return RN_OK;
}

int rn_server_poll(rn_server* s, int64_t* done_ids, int32_t max_ids, int32_t* n_done) {
  if (!s || !n_done || max_ids < 0 || (max_ids > 0 && !done_ids)) return RN_E_INVALID_ARG;
  std::lock_guard<std::mutex> lock(s->mu);
  progress(s);
  int32_t n = 0;
  for (auto& kv : s->jobs) {
    Job* j = kv.second.get();
    if (n >= max_ids) break;
    if (j->state == kDone && !j->reported) {
      j->reported = true;
      done_ids[n++] = j->id;
    }
  }
  *n_done = n;
  return RN_OK;
}

int rn_server_fetch(rn_server* s, int64_t job_id, int32_t* out, uint64_t* stats) {
  if (!s) return RN_E_INVALID_ARG;
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return RN_E_INVALID_ARG;
  Job* j = it->second.get();
  if (j->state == kQueued) return RN_E_INVALID_ARG;
  if (j->state == kRunning) {
    const hipError_t e = hipEventSynchronize(j->done);
    if (e != hipSuccess) return rn_internal::device_status(e);
    progress(s);
  }
  int rc = j->rc;
  const size_t out_bytes = (size_t)j->S * j->N * j->T * sizeof(int32_t);
  const size_t stats_bytes = (size_t)j->T * 4 * sizeof(uint64_t);
  if (rc == RN_OK && j->pin_out) {  // the results are already in host memory
    const char* b = s->pin + j->pin_off;
    if (out) std::memcpy(out, b + j->o_out, out_bytes);
    if (stats) std::memcpy(stats, b + j->o_stats, stats_bytes);
  } else if (rc == RN_OK) {
    // Copy on the server's copy stream: the job's own stream may already run a
    // later job, and a copy queued behind it would wait for that kernel.
    hipStream_t st = s->copy;
    hipError_t e = hipSuccess;
    if (out)
      e = hipMemcpyAsync(out, s->base + j->off + j->o_out, out_bytes, hipMemcpyDeviceToHost, st);
    if (stats && e == hipSuccess)
      e = hipMemcpyAsync(stats, s->base + j->off + j->o_stats, stats_bytes,
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = rn_internal::device_status(e);
  }
  release_device(s, j);
  release_pinned(s, j);
  (void)hipEventDestroy(j->done);
  s->jobs.erase(it);
  progress(s);
  return rc;
}

int rn_server_status(rn_server* s, int64_t* queued, int64_t* running, int64_t* bytes_in_use) {
  if (!s) return RN_E_INVALID_ARG;
  std::lock_guard<std::mutex> lock(s->mu);
  if (queued) *queued = (int64_t)s->queue.size();
  if (running) *running = s->running;
  if (bytes_in_use) *bytes_in_use = (int64_t)s->in_use;
  return RN_OK;
}

void rn_server_free(rn_server* s) {
  if (!s) return;
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& kv : s->jobs)
    if (kv.second->done) (void)hipEventDestroy(kv.second->done);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  if (s->copy) (void)hipStreamDestroy(s->copy);
  if (s->base) (void)hipFree(s->base);
  if (s->pin) (void)hipHostFree(s->pin);
  delete s;
}

}  // extern "C"
