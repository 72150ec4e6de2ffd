/*
 * oracle.h -- plain FP64 CPU oracle for tau-leaping parameter sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path; it is
 * loaded by the test suite, by the package's smoke check and by the benchmark's
 * CPU-baseline leg, and by nothing else.  It shares no source, header, table or
 * helper with the HIP path.
 *
 * What it computes: independent sample paths of the continuous-time Markov
 * chain X(t) of molecule counts (paper, Methods section), advanced by the
 * Cao-Gillespie-Petzold tau-leaping method with critical-reaction handling and
 * exact-SSA fallback (Y. Cao, D. T. Gillespie, L. R. Petzold, J. Chem. Phys.
 * 124, 044109 (2006); critical reactions from J. Chem. Phys. 123, 054104
 * (2005); the exact steps are Gillespie's direct method, J. Phys. Chem. 81,
 * 2340 (1977)).  Random numbers come from Philox4x32-10 (Salmon, Moraes,
 * Dror, Shaw, SC'11) and Poisson variates from sequential inversion (small
 * means) or Hoermann's PTRS (Insurance: Math. & Econ. 12 (1993) 39).
 */
#ifndef RN_ORACLE_H
#define RN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_species, n_reactions;
  const int32_t *react_ptr, *react_species, *react_coeff; /* CSR, n_reactions+1 offsets */
  const int32_t *prod_ptr, *prod_species, *prod_coeff;
} orc_net_desc;

typedef struct {
  uint64_t seed;
  double eps;          /* leap-condition tolerance epsilon                         */
  int32_t n_c;         /* critical threshold: L_j < n_c makes reaction j critical   */
  double ssa_factor;   /* leap only when tau' >= ssa_factor / a0                    */
  int32_t ssa_burst;   /* exact events run when the switch trips                    */
  uint64_t max_steps;  /* per trajectory: leaps + ssa events + rejections           */
  int32_t method;      /* 0 = tau-leaping, 1 = exact SSA only                        */
  double cle_threshold; /* > 0: leap firings with mean >= this are Gaussian (CLE)    */
} orc_params;

/* Counts of primitive operations, summed over the trajectories of one call. */
typedef struct {
  uint64_t leaps, ssa_events, rejections;
  uint64_t prop_evals;      /* a_j evaluations                                    */
  uint64_t crit_tests;      /* consumed-species tests in the critical rule        */
  uint64_t tau_terms;       /* (species, reaction) terms of mu/sigma^2             */
  uint64_t tau_species;     /* species bounds evaluated                            */
  uint64_t philox_blocks;   /* distinct Philox4x32-10 blocks consumed              */
  uint64_t inv_draws, inv_iters;    /* inversion draws and their loop iterations  */
  uint64_t ptrs_draws, ptrs_iters, ptrs_log_tests;
  uint64_t exp_draws;       /* exponential waiting times                           */
  uint64_t select_terms;    /* terms scanned by the reaction-selection searches    */
  uint64_t update_terms;    /* stoichiometry entries applied                       */
} orc_ops;

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* 53-bit uniform on [0,1) from the word pair (hi, lo). */
double orc_u53(uint32_t hi, uint32_t lo);
/* One Poisson(lam) variate for reaction j of attempt n of trajectory traj. */
int64_t orc_poisson(double lam, uint64_t seed, uint32_t traj, uint32_t n, int32_t j,
                    orc_ops *ops);

/* Chemical-Langevin firing count for mean lam (>= 10): round(lam + sqrt(lam) z),
 * z standard normal by Box-Muller, floored at 0 and clamped at 2^31. */
int64_t orc_cle_count(double lam, uint64_t seed, uint32_t traj, uint32_t n, int32_t j);
void orc_cle_many(double lam, uint64_t seed, uint32_t n0, int32_t j, int64_t n, int64_t *out);

/* n variates for trajectory ids 0..n-1 (test helper). */
void orc_poisson_many(double lam, uint64_t seed, uint32_t n0, int32_t j, int64_t n, int64_t *out);

/* Test hooks for the two decisions whose ties no trajectory statistic can see:
 * the direct method's selection over propensities a[0..m) (allowed may be
 * NULL), and the critical race (1 when a critical reaction fires). */
int orc_pick_index(const double *a, int m, double r, const int *allowed);
int orc_critical_fires(double tau_c, double tau_p, double delta);

/* Status bits of a trajectory. */
#define ORC_ST_ABSORBED 1u
#define ORC_ST_MAXSTEPS 2u
#define ORC_ST_OVERFLOW 4u

/* Error codes. */
#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NET (-2)
#define ORC_E_ORDER (-3)
#define ORC_E_NOMEM (-4)

/*
 * Simulate n_traj trajectories with global ids traj_first .. traj_first+n_traj-1.
 *   rates : rates[j*rates_ld + t]  (t = local trajectory index)
 *   x0    : x0[i] when x0_ld == 0, else x0[i*x0_ld + t]
 *   times : S strictly increasing, non-negative sample times
 *   out   : out[(s*N + i)*out_ld + t]
 *   stats : stats[t*4 + {0: leaps, 1: ssa events, 2: rejections, 3: status}]
 *   ops   : optional operation counters (may be NULL)
 */
int orc_run(const orc_net_desc *net, const double *rates, int64_t rates_ld,
            const int32_t *x0, int64_t x0_ld, const double *times, int32_t n_times,
            int64_t traj_first, int64_t n_traj, int32_t *out, int64_t out_ld,
            uint64_t *stats, const orc_params *par, orc_ops *ops);

/*
 * Deterministic counterpart (paper, Methods section: when every species is
 * abundant, X(t) is well approximated by the reaction-rate equations, and the
 * thermodynamic limit makes the stochastic and mean-field models agree):
 *   dy/dt = sum_j nu_j c_j h_j(y),  h_j = 1, y_a, y_a*y_b, or y_a^2/2 (homodimer),
 * integrated with the Dormand-Prince 5(4) embedded Runge-Kutta pair, or with a
 * Rosenbrock 4(3) method for stiff networks, under an error-per-step
 * controller; steps are clipped to the sample times.
 *   out   : out[(s*N + i)*out_ld + t] (double)
 *   stats : stats[t*4 + {0: accepted steps, 1: rejected steps, 2: 0, 3: status}]
 */
typedef struct {
  double rtol, atol;
  uint64_t max_steps;  /* accepted + rejected steps per trajectory */
  int32_t method;      /* ORC_ODE_DOPRI5 or ORC_ODE_ROS4 */
} orc_ode_params;

/* Integrators of orc_ode_run: the explicit Dormand-Prince 5(4) pair, or the
 * linearly implicit Rosenbrock 4(3) method for stiff networks (its
 * construction is described at the top of ode.c). */
#define ORC_ODE_DOPRI5 0
#define ORC_ODE_ROS4 1

int orc_ode_run(const orc_net_desc *net, const double *rates, int64_t rates_ld,
                const int32_t *x0, int64_t x0_ld, const double *times, int32_t n_times,
                int64_t n_traj, double *out, int64_t out_ld, uint64_t *stats,
                const orc_ode_params *par);

/*
 * Hybrid stochastic/deterministic sweep (a piecewise-deterministic Markov
 * process; the construction is described at the top of ode.c).  cont[j] != 0
 * makes reaction j continuous (part of the flow), 0 discrete (a jump).
 * Trajectory t of the call has the Philox id traj0 + t.
 *   out   : out[(s*N + i)*out_ld + t] (double); samples take the pre-jump state
 *   stats : stats[t*4 + {0: accepted steps, 1: rejected steps and jump-location
 *           trials, 2: jumps, 3: status}]
 */
typedef struct {
  uint64_t seed;
  double rtol, atol;
  uint64_t max_steps;  /* accepted + rejected steps per trajectory (checked per step) */
} orc_hybrid_params;

int orc_hybrid_run(const orc_net_desc *net, const int32_t *cont, const double *rates,
                   int64_t rates_ld, const int32_t *x0, int64_t x0_ld, const double *times,
                   int32_t n_times, int64_t traj0, int64_t n_traj, double *out, int64_t out_ld,
                   uint64_t *stats, const orc_hybrid_params *par);

#ifdef __cplusplus
}
#endif
#endif
