// rn_kernel.h -- packed device tables and kernel parameters of the sweep kernels.
//
// Internal to the library (host code in rn_host.cpp fills these, the kernels in
// rn_sweep_kernel.h, rn_ode.hip and rn_moments.hip read them).  Every table is read with wave-uniform indices, so the
// kernels fetch them through the scalar data cache.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

namespace rn {

// One reaction's rate law: a_j = c_j * s_j * (x[ia] * (x[ib] + db)), where the
// pseudo-species N always holds 1 (so order 0 uses ia = ib = N, order 1 uses
// ib = N), a homodimer uses ib = ia, db = -1, s_j = 1/2, and every other case
// has db = 0, s_j = 1.
struct RateLaw {
  int32_t ia, ib, db, dimer;
};

// Leap-condition entry of one reactant species (CGP 2006): its species index,
// the g-rule (1: highest order 1; 2: highest order 2, never two molecules of it
// in one reaction; 3: highest order 2 with a homodimer), and its range in the
// species-major stoichiometry list.
struct TauSpecies {
  int32_t species, gkind, begin, end;
};

struct DevNet {
  // M counts the null reactions (zero rate, no stoichiometry) that pad the
  // network to a whole number of 16-reaction rate vectors; M_real does not.
  int32_t N, M, M_real, n_rs, crit_words;
  const RateLaw* law;        // [M]
  const int32_t* nu_ptr;     // [M+1] reaction-major net changes
  const int2* nu_ent;        // {species, nu_ij}, nu_ij != 0
  const int32_t* cons_ptr;   // [M+1] consumed reactants (nu_ij < 0)
  const int2* cons_ent;      // {species, |nu_ij|}
  const uint32_t* nu_abs;    // [M] sum_i |nu_ij|
  const TauSpecies* rs;      // [n_rs] reactant species, ascending
  const int2* rs_ent;        // {j, nu_ij} per reactant species, ascending j
  const int32_t* col_ptr;    // [N+1] species-major net changes (all species)
  const int2* col_ent;       // {j, nu_ij}, ascending j
  const double* log_fact;    // [kLogFactTable] log(k!) for small k
  const int32_t* nu_dense;   // [M_real][row stride] dense nu_ij (network-compiled kernels), or null
};

constexpr int kLogFactTable = 1024;

struct SweepParams {
  DevNet net;
  const double* rates;
  int64_t rates_ld;
  const int32_t* x0;
  int64_t x0_ld;
  const double* times;
  int32_t n_times;
  int32_t* out;
  int64_t out_ld;
  uint64_t* stats;
  int64_t n_traj;
  uint32_t traj_offset;
  uint32_t key0, key1;
  double eps;
  int32_t n_c;
  double ssa_factor;
  int32_t ssa_burst;
  uint64_t max_steps;
  int32_t method;
  double cle_threshold;  // 0: off
  // Leap-side phases run when at least this fraction of the wave's active lanes
  // waits for them (or no lane is in an SSA burst).  Scheduling only: results do
  // not depend on it.
  float theta;
  uint64_t* phase_cycles;  // optional per-wave phase profile (network-compiled kernel)
  // Fused ensemble statistics (null: off).  During the sweep sum_x2 holds, per
  // (sample, species), the sums of the low and of the high 32-bit words of
  // x^2; a finishing pass turns them into the 128-bit sum.
  uint64_t* sum_x;     // [n_times * N]
  uint64_t* sum_x2;    // [n_times * N][2]
  uint32_t* hist;      // [n_times * N][hist_bins]
  const int32_t* hist_lo;     // [N]
  const int32_t* hist_width;  // [N]
  int32_t hist_bins;
  int32_t out_traj_major;     // 0: out[(s * N + i) * out_ld + t]; 1: out[t * out_ld + s * N + i]
};

// Reaction-rate-equation sweep (Dormand-Prince 5(4) per lane).
constexpr int kOdeSlots = 10;  // state vectors per lane in the workspace

struct OdeParams {
  DevNet net;
  const double* rates;
  int64_t rates_ld;
  const int32_t* x0;
  int64_t x0_ld;
  const double* times;
  int32_t n_times;
  double* out;
  int64_t out_ld;
  uint64_t* stats;
  double* work;
  int64_t work_ld;
  int64_t n_traj;
  double rtol, atol;
  uint64_t max_steps;
};

// Hybrid (piecewise-deterministic) sweep: continuous reactions form a flow
// integrated like the rate equations, discrete ones jump.
constexpr int kHybridSlots = 12;  // state vectors per lane in the workspace

struct HybridParams {
  DevNet net;
  const int32_t* cont;  // [M_real]: nonzero = continuous
  const double* rates;
  int64_t rates_ld;
  const int32_t* x0;
  int64_t x0_ld;
  const double* times;
  int32_t n_times;
  double* out;
  int64_t out_ld;
  uint64_t* stats;
  double* work;
  int64_t work_ld;
  int64_t n_traj;
  uint32_t traj_offset;
  uint32_t key0, key1;
  double rtol, atol;
  uint64_t max_steps;
};

// A device work queue of sweep blocks for the persistent batch kernel: item k
// is (job, block) = items[2k], items[2k + 1], block b of a job covering its
// trajectories [b * WG, (b + 1) * WG).  `next` counts the items taken; it is
// zero when the kernel starts.
struct BatchQueue {
  const SweepParams* jobs;
  const int32_t* items;
  int32_t n_items;
  uint32_t* next;
};

#ifndef __HIPCC_RTC__
// Launch configuration chosen by the host.
struct LaunchCfg {
  int wg;          // lanes (= trajectories) per workgroup: 64 or 256
  int rate_segs;   // 0: rates read from memory; k: held in k register vectors of 16
  size_t lds_bytes;
};

// Kernel LDS bytes per lane: two count buffers of N+1 words and the
// critical-reaction bit words.
constexpr int kMaxRateSegs = 8;

inline size_t lds_words_per_lane(int N, int M) {
  return 2 * (size_t)(N + 1) + (size_t)((M + 31) / 32);
}

hipError_t launch_sweep_f64(const SweepParams& p, const LaunchCfg& cfg, hipStream_t stream);
hipError_t launch_sweep_f32(const SweepParams& p, const LaunchCfg& cfg, hipStream_t stream);
// Persistent batch kernels (rn_sweep_f64.hip, rn_sweep_f32.hip): `groups`
// workgroups take items of q until it is empty; cfg gives the workgroup size,
// the rate registers and the LDS bytes (at least every job's).
hipError_t launch_persistent_f64(const BatchQueue& q, const LaunchCfg& cfg, hipStream_t stream,
                                 int64_t groups);
hipError_t launch_persistent_f32(const BatchQueue& q, const LaunchCfg& cfg, hipStream_t stream,
                                 int64_t groups);
hipError_t launch_ode(const OdeParams& p, hipStream_t stream);
// Workspace of the allocation-free rate-equation sweep: a file-scope device
// array of kOdeScratchDoubles doubles per device (32 MiB), whose address on the
// current device ode_scratch returns (resolved once per device).
constexpr int64_t kOdeScratchDoubles = (int64_t)4 << 20;
constexpr int kMaxDevices = 64;
hipError_t ode_scratch(double** ptr);
// Rosenbrock 4(3) rate-equation sweep (rn_ros.hip): one wave per trajectory;
// ros_fits says whether a network fits it (at most 64 species, W in LDS).
bool ros_fits(int n_species, int m_real);

// The one-wave-per-trajectory sweep (rn_wsweep.hip): networks of at most
// kWsweepMaxSpecies species and kWsweepMaxReactions reactions.
constexpr int kWsweepMaxSpecies = 512, kWsweepMaxReactions = 512;
bool wsweep_fits(int n_species, int m_real);
// Dynamic LDS of its 64-lane workgroup.
size_t wsweep_lds_bytes(int n_species, int m_real, bool fp32);
// Enqueue it: one workgroup per trajectory of p (p.net.M_real <= 512); n_simd:
// the device's SIMDs (4 per CU), which picks the occupancy of the largest form.
hipError_t launch_wsweep(const SweepParams& p, bool fp32, int n_simd, hipStream_t stream);
hipError_t launch_ros(const OdeParams& p, hipStream_t stream);
hipError_t launch_hybrid(const HybridParams& p, hipStream_t stream);
hipError_t launch_moments(const int32_t* out, int64_t out_ld, int64_t rows, int64_t n_traj,
                          int64_t* sum_x, uint64_t* sum_x2, hipStream_t stream);
// Fused statistics of a sweep: zero the arrays before it, and afterwards turn
// the split word sums of x^2 into 128-bit sums (rn_moments.hip).
hipError_t launch_stats_zero(const SweepParams& p, hipStream_t stream);
hipError_t launch_stats_finish(const SweepParams& p, hipStream_t stream);
// p[0 .. n) = v, by a kernel (rn_moments.hip).
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);
#endif  // __HIPCC_RTC__

}  // namespace rn
