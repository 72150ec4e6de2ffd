/*
 * rn.h -- C ABI of the MI355X (gfx950) tau-leaping parameter-sweep library.
 *
 * The library runs many independent stochastic simulations of one mass-action
 * reaction network, one per parameterization (kinetic constants and initial
 * amounts differ between simulations: paper, Aims and motivation section).  The
 * state of a simulation is the vector of molecule counts per species, and a
 * reaction firing changes it by the reaction's stoichiometry (paper, Methods
 * section).  Each simulation is advanced by Cao-Gillespie-Petzold tau-leaping
 * (Y. Cao, D. T. Gillespie, L. R. Petzold, J. Chem. Phys. 124, 044109 (2006))
 * with critical reactions (J. Chem. Phys. 123, 054104 (2005)) and bursts of
 * exact SSA events (Gillespie, J. Phys. Chem. 81, 2340 (1977)).
 *
 * Conventions
 *  - Every function returns RN_OK (0) or a negative RN_E_* code, except
 *    rn_free_network (void) and rn_strerror (string).
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the device that was current when the network was loaded.
 *  - Nothing here takes or returns a framework type; all sizes are int32/int64.
 */
#ifndef RN_H
#define RN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RN_OK 0
#define RN_E_INVALID_ARG (-1)     /* null pointer, bad size, bad option                 */
#define RN_E_INVALID_NETWORK (-2) /* species index out of range, coefficient <= 0 ...   */
#define RN_E_UNSUPPORTED (-3)     /* a reaction with three or more reactant molecules   */
#define RN_E_NOMEM (-4)           /* host or device allocation failed                   */
#define RN_E_DEVICE (-5)          /* a HIP call failed; rn_last_device_error() names it */
#define RN_E_SCRATCH (-6)         /* input exceeds the fixed scratch of a no-alloc call   */

/* Per-trajectory status bits (stats[t][3]); never a call error. */
#define RN_ST_ABSORBED 1u /* total propensity reached 0; later samples repeat the state     */
#define RN_ST_MAXSTEPS 2u /* leaps + SSA events + rejections reached max_steps              */
#define RN_ST_OVERFLOW 4u /* a count would exceed 2^31-1; later samples repeat the last state */

#define RN_METHOD_TAULEAP 0 /* CGP tau-leaping with critical reactions and SSA bursts */
#define RN_METHOD_SSA 1     /* exact SSA events only (Gillespie direct method)        */

#define RN_OUT_SAMPLE_MAJOR 0 /* out[(s * N + i) * out_ld + t] */
#define RN_OUT_TRAJ_MAJOR 1   /* out[t * out_ld + s * N + i]   */

#define RN_FP64 0 /* all of the method's arithmetic in double precision                  */
#define RN_FP32 1 /* single-precision propensities, SSA events, tau' and Poisson means;
                     double precision for time, the SSA-switch test and the critical race */

/*
 * Network description (host memory, caller-owned, copied by rn_load_network).
 * Reaction j has reactants react_species/coeff[react_ptr[j] .. react_ptr[j+1])
 * and products prod_species/coeff[prod_ptr[j] .. prod_ptr[j+1]) (compressed
 * rows, n_reactions+1 offsets each).  A species listed twice in one list has
 * its coefficients added.  Mass-action order (sum of reactant coefficients)
 * must be 0, 1 or 2; coefficients must lie in [1, 2^20].  A reaction may have no
 * products (degradation) or no reactants (source).
 */
typedef struct {
  int32_t n_species, n_reactions;
  const int32_t *react_ptr, *react_species, *react_coeff;
  const int32_t *prod_ptr, *prod_species, *prod_coeff;
} rn_network_desc;

typedef struct rn_network rn_network; /* opaque; immutable after load */

/*
 * Validate and preprocess a network (paper, Methods section: species counts and
 * the reactions that change them) and upload its tables to the current HIP
 * device.  On success *out owns a library handle (free with rn_free_network).
 * Errors: RN_E_INVALID_ARG (null pointer, n_species or n_reactions <= 0,
 * offsets not non-decreasing), RN_E_INVALID_NETWORK (species index out of
 * range, coefficient out of [1, 2^20]), RN_E_UNSUPPORTED (order > 2),
 * RN_E_NOMEM, RN_E_DEVICE.  *out is untouched on error.
 */
int rn_load_network(const rn_network_desc *desc, rn_network **out);

/* Release a handle and its device tables (null is ignored).  The caller must
 * make sure no sweep using it is still running.  Freeing device memory waits
 * for all work on the device (hipFree), so a serving loop frees handles when
 * the device is idle rather than after each job. */
void rn_free_network(rn_network *net);

/* Number of species / reactions of a loaded network (-1 for a null handle). */
int32_t rn_network_species(const rn_network *net);
int32_t rn_network_reactions(const rn_network *net);

/*
 * Equally spaced observation times of X(t) on [0, t_end] (paper, Methods
 * section: sample paths observed through time): out[s] = s * t_end / (n - 1)
 * for s < n-1 and out[n-1] = t_end exactly; n = 1 gives {t_end}.  `out` is a
 * host array of n_points doubles.  Errors: RN_E_INVALID_ARG when out is null,
 * n_points < 1, or t_end is negative or not finite.
 */
int rn_sample_times(double t_end, int32_t n_points, double *out);

/*
 * One parameter sweep: n_traj independent trajectories of the network, each
 * with its own rate constants (and optionally its own initial counts), all
 * observed at the same sample times.
 *
 *  traj_offset  global id of local trajectory 0; trajectory t draws from the
 *               Philox4x32-10 stream keyed by `seed` with counter word 0 equal
 *               to traj_offset + t, so a sweep split into ranges reproduces the
 *               unsplit one exactly.  traj_offset + n_traj <= 2^32.
 *  rates        device, double, rates[j * rates_ld + t] (reaction-major,
 *               trajectory-minor), rates_ld >= n_traj; finite and >= 0.
 *  x0           device, int32: x0[i] (x0_ld == 0, broadcast to every
 *               trajectory) or x0[i * x0_ld + t] (x0_ld >= n_traj); >= 0.
 *  times        device, double[n_times]; must be finite, >= 0 and strictly
 *               increasing (device memory is not inspected on the host; the
 *               Python binding checks it before upload).
 *  out          device, int32, receives X_i(times[s]) of trajectory t at
 *               out[(s * n_species + i) * out_ld + t] (out_layout
 *               RN_OUT_SAMPLE_MAJOR, the default; out_ld >= n_traj) or at
 *               out[t * out_ld + s * n_species + i] (RN_OUT_TRAJ_MAJOR;
 *               out_ld >= n_times * n_species).  May be null when fused
 *               statistics (sum_x, hist below) are requested.
 *  stats        device, uint64[n_traj][4]: accepted leaps, SSA events,
 *               rejected leaps, status bits (RN_ST_*).
 *  eps          leap-condition tolerance (finite, > 0); n_c critical threshold
 *               (0 <= n_c <= 2^20); ssa_factor: leap only when
 *               tau' >= ssa_factor / a0 (>= 0); ssa_burst: exact events per
 *               burst (>= 1); max_steps: per-trajectory cap on leaps + SSA
 *               events + rejections (>= 1).
 *  method       RN_METHOD_TAULEAP or RN_METHOD_SSA.
 *  precision    RN_FP64: every step in double precision (trajectories are a
 *               deterministic function of the inputs and the seed).
 *               RN_FP32: rates are rounded to float on load; propensities, the
 *               SSA event (a0, waiting time, selection), the leap-condition
 *               bound tau', the Poisson means and the small-mean inversion
 *               sampler run in float with 24-bit uniforms (the top 24 bits of
 *               the word pair that RN_FP64 uses for the same draw); time, the
 *               sample times, a0 of the SSA-switch test, the critical race
 *               (a0c, tau'' and its selection), the leap length and the PTRS and
 *               Langevin samplers stay in double.  The same seed gives the same
 *               random path in both modes until a float rounding changes a
 *               decision, so FP32 results agree with FP64 in distribution, not
 *               bit for bit.
 *
 * Buffers are caller-owned and must not overlap.  The call only validates the
 * arguments it can see on the host and enqueues kernels on `hip_stream` (a
 * hipStream_t; null = the default stream); it returns before they finish and
 * allocates nothing.  Per-trajectory conditions go to stats[t][3].  Errors:
 * RN_E_INVALID_ARG, RN_E_DEVICE.  Concurrent sweeps on one handle are allowed.
 */
typedef struct {
  int64_t n_traj;
  int64_t traj_offset;
  const double *rates;
  int64_t rates_ld;
  const int32_t *x0;
  int64_t x0_ld;
  const double *times;
  int32_t n_times;
  int32_t *out;
  int64_t out_ld;
  uint64_t *stats;
  uint64_t seed;
  double eps;
  int32_t n_c;
  double ssa_factor;
  int32_t ssa_burst;
  uint64_t max_steps;
  int32_t method;
  int32_t precision;
  /* 0 (off), or >= 10: a leap's firing count of a non-critical reaction whose
   * mean lam reaches this value is drawn from the Chemical Langevin increment
   * round(lam + sqrt(lam) z), z standard normal (Box-Muller on the reaction's
   * first PTRS block), floored at 0 -- the CLE-based approximation of the
   * paper's Methods section, in place of the Poisson draw. */
  double cle_threshold;
  /* Optional profile (null: off): device uint64 [ceil(n_traj / 64)][4], filled
   * per wave with the shader-clock cycles spent in SSA events, in the decide
   * phase, in leap attempts, and in total -- only by the network-compiled
   * kernel when the process environment sets RN_PHASE_TIMERS=1 (a separately
   * compiled kernel; the results are unchanged).  Otherwise left untouched. */
  uint64_t *phase_cycles;
  /* Fused ensemble statistics (all null: off), the summaries that parameter
   * sweeps, sensitivity analysis and parameter estimation consume (paper, Aims
   * and motivation section), accumulated by the sweep kernels as each
   * trajectory reaches each sample time, so that the [n_times][N][n_traj]
   * sample array need not be written (out may then be null):
   *  sum_x    device uint64 [n_times][N]: sum over the call's trajectories of
   *           X_i(times[s]) (exact);
   *  sum_x2   device uint64 [n_times][N][2]: the sum of X_i^2 as an unsigned
   *           128-bit integer (low word, high word; exact).  sum_x and sum_x2
   *           are given together.  Mean and variance follow as for rn_moments.
   *  hist     device uint32 [n_times][N][hist_bins]: counts of X_i(times[s])
   *           in bins of hist_width[i] molecules from hist_lo[i] (device int32
   *           [N] each, widths >= 1); bin b holds lo + b w <= x < lo + (b+1) w,
   *           counts below lo go to bin 0 and from lo + hist_bins w on to the
   *           last bin.  hist_bins >= 1 when hist is set (n_times * N *
   *           hist_bins < 2^31).
   * The call sets these arrays to zero before its trajectories run, on the
   * same stream; a sweep split into trajectory ranges adds the ranges' arrays.
   * Sums are exact integers, so they equal the sums of the sample array. */
  uint64_t *sum_x;
  uint64_t *sum_x2;
  uint32_t *hist;
  const int32_t *hist_lo;
  const int32_t *hist_width;
  int32_t hist_bins;
  /* RN_OUT_SAMPLE_MAJOR (0, default) or RN_OUT_TRAJ_MAJOR (1), the layout of
   * `out` above.  Trajectories reach the sample times at different moments,
   * so in the sample-major layout the 64 lanes of a wave write their values of
   * one (sample, species) row at different times, each store covering part of
   * a cache line; in the trajectory-major layout every trajectory writes its
   * own contiguous rows, whole lines in sequence. */
  int32_t out_layout;
} rn_sweep_args;

/* Defaults: eps 0.03, n_c 10, ssa_factor 10, ssa_burst 100, max_steps 1e8,
 * tau-leaping, FP64, CLE off (CGP 2006's recommended switch constants). */
void rn_sweep_args_init(rn_sweep_args *args);

int rn_sweep(const rn_network *net, const rn_sweep_args *args, void *hip_stream);

/*
 * Which kernel rn_sweep runs for this network, precision and n_traj.
 * Networks with at most 63 species and 128 reactions get a kernel compiled for
 * that network (hipRTC, on first use, then cached for the process): its counts,
 * rate constants and tables are compile-time values in registers, and it gives
 * the same results as the generic kernels, which run otherwise (also when the
 * environment sets RN_JIT=0 or the compilation fails).  The first rn_sweep of a
 * network and precision pays the compilation on the calling thread.  The
 * other networks of at most 512 species and 512 reactions run one wave per
 * trajectory (lanes over reactions and species), and so do sweeps of at most
 * 16 trajectories per compute unit on networks with a compiled kernel; the
 * remaining sweeps run one lane per trajectory.  RN_WSWEEP=1 picks the wave
 * form whenever the network fits it, RN_WSWEEP=0 never.  All kernels give the
 * same trajectories.
 * Returns 1 (network-compiled; compiling it now if needed), 0 (generic, one
 * lane per trajectory), 2 (generic, one wave per trajectory), or
 * RN_E_INVALID_ARG / RN_E_DEVICE.
 * When the environment sets RN_JIT_CACHE to a directory, compiled code objects
 * are also kept there (one file per network, precision and launch shape,
 * holding the complete compilation input beside the object; a file is used
 * only when its stored input equals the current one), so later processes skip
 * the compilation.
 */
int rn_sweep_kernel_kind(const rn_network *net, int32_t precision, int64_t n_traj);

/*
 * Drop the network-kernel compilations queued in the background (by
 * rn_server_submit) that have not started, and wait for those running.  The
 * dropped networks keep the generic kernel for the rest of the process.  Call
 * it before the process exits if a server was used: a compilation still
 * running while the process tears down its libraries can crash the exit.  The
 * Python binding registers it to run at interpreter exit.
 */
void rn_compile_drain(void);

/*
 * Batched sweeps: many jobs (each a network handle and an rn_sweep_args, e.g. a
 * set of networks of uneven size and trajectory count) launched together.  The
 * jobs are independent parameter sweeps (paper, Aims and motivation section);
 * the first rn_batch_launch records all of them into one HIP graph as parallel
 * branches (largest jobs first, spread over RN_BATCH_BRANCHES internal streams,
 * default 8; give the process at least as many hardware queues through
 * GPU_MAX_HW_QUEUES for them to run at once), and every later launch replays
 * that graph with one hipGraphLaunch on `hip_stream`.
 * Each job's results are exactly those of rn_sweep with the same arguments.
 *
 *  rn_batch_add   validates `args` like rn_sweep (and compiles the network's
 *                 kernel if needed), copies them; the buffers they point to
 *                 and the network handle must stay valid while the batch is
 *                 used.  Jobs cannot be added after the first launch
 *                 (RN_E_INVALID_ARG).  All jobs must be on one device.
 *  rn_batch_launch  asynchronous on `hip_stream`; a replay reads the inputs
 *                 and rewrites the outputs the buffers hold at that time.
 *  rn_batch_size  number of non-empty jobs, or RN_E_INVALID_ARG.
 * Errors: RN_E_INVALID_ARG, RN_E_NOMEM, RN_E_DEVICE, and those of rn_sweep.
 */
typedef struct rn_batch rn_batch;
int rn_batch_create(rn_batch **out);
/*
 * Persistent form of a batch (before its first launch; on = 0 restores the
 * graph of per-job kernels).  Every job runs the generic kernel body (the same
 * trajectories as rn_sweep), cut into blocks of one workgroup; the jobs that
 * share a launch shape (precision, trajectories per workgroup, rate constants
 * in registers or read from memory, and LDS footprint class) form one device
 * work queue of (job, block) items, largest jobs first, and one persistent
 * kernel per shape takes items until its queue is empty.  The kernels are the
 * branches of the graph that rn_batch_launch records and replays (after a
 * kernel node that zeroes the queue counters).  A job's shape comes from
 * rn_batch_tune when its bucket was tuned, else 64-lane workgroups with its
 * rates in registers when they fit.  The launch allocates the queues once, at
 * the first rn_batch_launch.  Errors: RN_E_INVALID_ARG (null, or after the
 * first launch).
 */
int rn_batch_persistent(rn_batch *b, int32_t on);
/*
 * Autotune the persistent form's launch shapes for the batch's jobs (before
 * its first launch).  Jobs are bucketed by (precision, species / 8, reactions
 * / 16, nonzero stoichiometry entries / 32); for every bucket not yet tuned in
 * this process, the bucket's largest job is timed on `hip_stream` in short
 * trials (up to 256 trajectories per compute unit, each stopped after 400
 * steps) for every candidate: 64 or 256 trajectories per workgroup, rate
 * constants in registers or in memory, and wave-scheduling thresholds 0.35,
 * 0.5, 0.65 (the fraction of a wave's live lanes that must wait for a leap
 * before the leap phases run); the fastest is kept.  Trials write into the
 * job's own output and stats arrays (a launch rewrites them) and never touch
 * its fused statistics.  Choices persist for the process and, when the
 * environment sets RN_TUNE_CACHE to a file path, are read from and written to
 * that file; RN_TUNE_LOG=1 prints one line per tuned bucket on stderr.
 * Synchronous; allocates temporary device memory.  Errors: RN_E_INVALID_ARG,
 * RN_E_DEVICE.
 */
int rn_batch_tune(rn_batch *b, void *hip_stream);
int rn_batch_add(rn_batch *b, const rn_network *net, const rn_sweep_args *args);
int rn_batch_size(const rn_batch *b);
int rn_batch_launch(rn_batch *b, void *hip_stream);
void rn_batch_free(rn_batch *b);

/*
 * Sweep-job server: jobs of different networks and sizes admitted continuously
 * into a fixed HBM budget (many parameter sweeps in flight at once: paper, Aims
 * and motivation section).  rn_server_create allocates the budget once as an
 * arena, and a pinned host staging area of min(budget / 4, 4 GiB); each job
 * holds one block of the arena (inputs, samples, stats) from admission until
 * it completes when the staging area had room for the whole job (its results
 * are then copied there on the job's stream), else until its results are
 * fetched.  Jobs are admitted in submission order as soon as a block and one of
 * `max_running` stream slots are free, so jobs submitted while others run
 * overlap on the device.  Streams beyond the process's hardware queues
 * (GPU_MAX_HW_QUEUES) share queues and wait for each other's work: keep
 * max_running a few below it (the null stream, the library's upload stream and
 * the server's copy stream take one each).  Work advances inside the calls
 * (there is no server thread): call rn_server_poll regularly.  Submission starts
 * compiling the job's network kernel in the background (a few worker threads);
 * the job uses it if it is ready when the job is admitted, else the generic
 * kernel (same results).
 * Each job's results equal those of rn_sweep with the same inputs and options.
 *
 *  rn_serve_job   host inputs, copied at submission (the caller may free them
 *                 on return); `params` supplies seed, eps, n_c, ssa_factor,
 *                 ssa_burst, max_steps, method, precision and cle_threshold (its
 *                 pointer, size and stride fields are ignored).  The network
 *                 handle must stay valid until the job is fetched.
 *  rn_server_submit   queues the job and returns its id; RN_E_NOMEM if the job
 *                 alone exceeds the budget, RN_E_INVALID_ARG for bad inputs.
 *  rn_server_poll     admits and launches what fits, then reports up to
 *                 max_ids finished job ids (each once).
 *  rn_server_fetch    copies a finished (or running: it waits) job's samples
 *                 [n_times][N][n_traj] and stats [n_traj][4] to host buffers
 *                 (either may be null) and releases its memory;
 *                 RN_E_INVALID_ARG for an unknown or still-queued job.
 *  rn_server_status   queued and running job counts, bytes of the budget held.
 *  rn_server_free     waits for running jobs and releases everything.
 */
typedef struct rn_server rn_server;
typedef struct {
  const rn_network *net;
  int64_t n_traj;
  const double *rates; /* host, [M][n_traj] */
  const int32_t *x0;   /* host, [N], or [N][n_traj] when x0_per_traj != 0 */
  int32_t x0_per_traj;
  const double *times; /* host, [n_times]: finite, >= 0, strictly increasing */
  int32_t n_times;
  rn_sweep_args params;
} rn_serve_job;
int rn_server_create(int64_t hbm_budget_bytes, int32_t max_running, rn_server **out);
int rn_server_submit(rn_server *s, const rn_serve_job *job, int64_t *job_id);
int rn_server_poll(rn_server *s, int64_t *done_ids, int32_t max_ids, int32_t *n_done);
int rn_server_fetch(rn_server *s, int64_t job_id, int32_t *out, uint64_t *stats);
int rn_server_status(rn_server *s, int64_t *queued, int64_t *running, int64_t *bytes_in_use);
void rn_server_free(rn_server *s);

#define RN_ODE_DOPRI5 0 /* explicit Dormand-Prince 5(4) pair                            */
#define RN_ODE_ROS4 1   /* linearly implicit Rosenbrock 4(3) method, for stiff networks */

/*
 * Deterministic sweep: the reaction-rate equations that abundant species follow
 * (paper, Methods section: mean-field ODEs, which agree with the stochastic
 * model in the thermodynamic limit),
 *   dy/dt = sum_j nu_j c_j h_j(y),  h_j = 1, y_a, y_a*y_b, or y_a^2/2 (homodimer),
 * one trajectory per parameterization, from y(0) = x0, integrated by the
 * Dormand-Prince 5(4) pair with error control (rms over species of
 * e_i / (atol + rtol * max(|y_i|, |y_i'|)) <= 1) and steps ending exactly on
 * the sample times.
 *
 *  rates, x0, times  as for rn_sweep (device; rates_ld, x0_ld likewise).
 *  out        device, double, out[(s * n_species + i) * out_ld + t] = y_i(times[s]).
 *  stats      device, uint64[n_traj][4]: accepted steps, rejected steps, 0,
 *             status (RN_ST_MAXSTEPS when accepted + rejected reach max_steps;
 *             later samples repeat the last state).
 *  work       device scratch of 10 * n_species rows of work_ld doubles
 *             (work_ld >= n_traj; rn_ode_work_doubles gives the total for
 *             work_ld = n_traj), caller-owned; its contents on entry are ignored.
 *             Networks of up to 64 species run one wave per trajectory with
 *             the state in registers and leave it untouched (their sums over
 *             species then add in a butterfly order, not in species order).
 *  rtol, atol finite, > 0; max_steps >= 1.
 * Asynchronous on `hip_stream`; allocates nothing.  Errors: RN_E_INVALID_ARG,
 * RN_E_DEVICE.
 */
typedef struct {
  int64_t n_traj;
  const double *rates;
  int64_t rates_ld;
  const int32_t *x0;
  int64_t x0_ld;
  const double *times;
  int32_t n_times;
  double *out;
  int64_t out_ld;
  uint64_t *stats;
  double *work;
  int64_t work_ld;
  double rtol, atol;
  uint64_t max_steps;
  /* RN_ODE_DOPRI5 (default) or RN_ODE_ROS4: the Rosenbrock 4(3) method of
   * L. F. Shampine, ACM Trans. Math. Softw. 8 (1982) 93 (gamma = 1/2), in the
   * transformed form of Hairer and Wanner (Solving ODEs II, Sec. IV.7).  Each
   * step forms the exact Jacobian J of the rate equations at y, factors
   * W = I/(gamma h) - J by Gaussian elimination with partial pivoting and
   * solves four linear systems; it is stable on stiff networks (rates spanning
   * many decades), where the explicit pair needs steps of the fastest time
   * scale.  Error norm, controller (exponent -1/4) and sample clipping as
   * above; stats[t][1] counts rejected steps.  Networks of up to 64 species
   * (one wave per trajectory, W in LDS); others return RN_E_UNSUPPORTED.
   * `work` is not used. */
  int32_t method;
} rn_ode_args;

/* Defaults: rtol 1e-6, atol 1e-6, max_steps 1e7, RN_ODE_DOPRI5. */
void rn_ode_args_init(rn_ode_args *args);

/* Doubles of workspace rn_ode_sweep needs for n_traj trajectories with
 * work_ld = n_traj (-1 for a null handle or a negative n_traj). */
int64_t rn_ode_work_doubles(const rn_network *net, int64_t n_traj);

int rn_ode_sweep(const rn_network *net, const rn_ode_args *args, void *hip_stream);

/*
 * rn_ode_sweep without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * rn_ode_sweep; args->work and args->work_ld are ignored.  Where rn_ode_sweep
 * would run the lane kernel on `work` (networks of more than 64 species, or
 * too many reactions for the wave kernel's LDS), this call uses a fixed
 * scratch array of 32 MiB that the library holds on each device it runs on
 * until the process ends; it needs 10 * n_species doubles per trajectory, so
 * at most rn_ode_noalloc_max_traj(net) trajectories fit, and a larger n_traj
 * returns RN_E_SCRATCH with nothing enqueued.  The call performs no device or
 * host allocation of its own (the first call on a device resolves the
 * scratch's address).  Every call on one device shares that device's scratch:
 * calls that overlap on one device (different streams, or different host
 * threads) race, and the caller must order them.  Errors: those of
 * rn_ode_sweep, and RN_E_SCRATCH.
 */
int rn_ode_sweep_noalloc(const rn_network *net, const rn_ode_args *args, void *hip_stream);

/* Largest n_traj rn_ode_sweep_noalloc accepts for this network (2^32 when it
 * needs no scratch), or -1 for a null handle. */
int64_t rn_ode_noalloc_max_traj(const rn_network *net);

/*
 * Hybrid stochastic/deterministic sweep: a piecewise-deterministic Markov
 * process per trajectory (paper, Methods section: abundant species follow the
 * mean-field equations, low-amount species keep their fluctuations).
 * `continuous` (device, [n_reactions] int32, caller-owned) marks each reaction:
 *  - nonzero: continuous.  Between jumps the state follows the rate equations
 *    of these reactions, dy/dt = sum_j nu_j c_j h_j(y) with the h of
 *    rn_ode_sweep, integrated by the same Dormand-Prince 5(4) controller.
 *  - zero: discrete.  Reaction j jumps (y += nu_j) with intensity
 *    max(0, c_j h_j(y)), h_j = 1, y_a, y_a*y_b or y_a*(y_a-1)/2.  Jumps come
 *    when the intensity integral since the previous jump, integrated with the
 *    flow, reaches an Exp(1) draw (Salis and Kaznessis, J. Chem. Phys. 122,
 *    054103 (2005)); the crossing is searched by the Illinois regula falsi to
 *    |L - xi| <= 1e-12 (1 + xi) (at most 30 trials per jump).  The jumping
 *    reaction is the first discrete j with u * a0_D < a_1 + ... + a_j.
 * Jump k of trajectory traj_offset + t draws from Philox4x32-10 block
 * (traj_offset + t, k, 0, 2^31) keyed by `seed`: words 0-1 give
 * xi = -log(1 - u53), words 2-3 give u.  With every reaction continuous the
 * results are rn_ode_sweep's; with every reaction discrete, the direct
 * method's.
 *  out        device, [n_times][N][out_ld] doubles; samples take the state
 *             before a jump that lands exactly on them.
 *  stats      device, [n_traj][4] uint64: accepted steps, rejected steps and
 *             jump-search trials, jumps, status (2 = max_steps reached; the
 *             remaining samples repeat the last state).
 *  work       device scratch of 12 * n_species rows of work_ld doubles
 *             (rn_hybrid_work_doubles gives the total for work_ld = n_traj).
 *             Networks of up to 64 species run one wave per trajectory with
 *             the state in registers and leave it untouched; their sums over
 *             species add in a butterfly order rather than in species order.
 *  rtol, atol finite, > 0; max_steps >= 1 (accepted + rejected, checked
 *             before each step).
 * Asynchronous on `hip_stream`; allocates nothing.  Errors: RN_E_INVALID_ARG,
 * RN_E_DEVICE.
 */
typedef struct {
  int64_t n_traj;
  int64_t traj_offset;
  const int32_t *continuous;
  const double *rates;
  int64_t rates_ld;
  const int32_t *x0;
  int64_t x0_ld;
  const double *times;
  int32_t n_times;
  double *out;
  int64_t out_ld;
  uint64_t *stats;
  double *work;
  int64_t work_ld;
  uint64_t seed;
  double rtol, atol;
  uint64_t max_steps;
} rn_hybrid_args;

/* Defaults: rtol 1e-6, atol 1e-6, max_steps 1e7, seed 0, offset 0. */
void rn_hybrid_args_init(rn_hybrid_args *args);

/* Doubles of workspace rn_hybrid_sweep needs for n_traj trajectories with
 * work_ld = n_traj (-1 for a null handle or a negative n_traj). */
int64_t rn_hybrid_work_doubles(const rn_network *net, int64_t n_traj);

int rn_hybrid_sweep(const rn_network *net, const rn_hybrid_args *args, void *hip_stream);

/*
 * Ensemble moments of a sweep's samples, the summary that parameter sweeps,
 * sensitivity analysis and parameter estimation consume (paper, Aims and
 * motivation section).  For every sample s < n_times and species i < n_species,
 * over trajectories t < n_traj of out[(s * n_species + i) * out_ld + t]:
 *   sum_x[s * n_species + i]              = sum_t x         (int64, exact)
 *   sum_x2[2 * (s * n_species + i) + 0/1] = sum_t x^2       (unsigned 128-bit:
 *                                           low word, high word; exact)
 * Mean and unbiased variance follow as m = S1/T and (S2 - S1^2/T)/(T - 1).
 * `out` is the int32 sample array of rn_sweep (device); sum_x and sum_x2 are
 * caller-owned device arrays of n_times*n_species int64 and 2*n_times*n_species
 * uint64.  Asynchronous on `hip_stream`; allocates nothing.  Errors:
 * RN_E_INVALID_ARG (null pointer, non-positive size, out_ld < n_traj,
 * n_times * n_species >= 2^31), RN_E_DEVICE.
 */
int rn_moments(const int32_t *out, int64_t out_ld, int32_t n_times, int32_t n_species,
               int64_t n_traj, int64_t *sum_x, uint64_t *sum_x2, void *hip_stream);

/* Message for an RN_* code (static storage). */
const char *rn_strerror(int code);

/* The hipError_t of the most recent RN_E_DEVICE in this thread (0 if none). */
int rn_last_device_error(void);

#ifdef __cplusplus
}
#endif
#endif
