/*
 * oracle.c -- plain FP64 CPU oracle for tau-leaping parameter sweeps.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg.  Shares nothing with the HIP path.
 *
 * Scalar, one trajectory at a time, in the order the method states its steps,
 * with dense per-reaction loops; nothing is blocked, fused or reordered.  Built
 * with -O2 -ffp-contract=off so that every floating-point operation written here
 * is rounded exactly once, in the order written.
 *
 * Problem (paper, Methods section): X(t) is the vector of molecule counts; a
 * reaction firing changes it by its stoichiometric vector; X(t) is a
 * continuous-time Markov chain whose law is the chemical master equation, and
 * sample paths are drawn instead of solving it.  Many simulations differ only in
 * kinetic constants and initial amounts (Aims and motivation section).
 *
 * Method: Cao-Gillespie-Petzold tau-leaping (J. Chem. Phys. 124, 044109,
 * 2006): species-based leap condition with the g_i factors, critical reactions
 * (J. Chem. Phys. 123, 054104, 2005) handled by one exact firing, rejection
 * with halving of tau' when a count would go negative, and a switch to a burst
 * of exact SSA events (Gillespie 1977, direct method) when tau' is only a few
 * times 1/a0.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Random numbers                                                            */
/* ------------------------------------------------------------------------- */

/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 Philox
 * S-box with multipliers 0xD2511F53, 0xCD9E8D57 and the Weyl key schedule
 * 0x9E3779B9, 0xBB67AE85; round r uses key + r * schedule. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* u = floor(((hi << 32) | lo) / 2^11) * 2^-53, in [0, 1). */
double orc_u53(uint32_t hi, uint32_t lo) {
  uint64_t z = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
  return (double)z * 0x1p-53;
}

/* Counter layout: (trajectory id, attempt/event counter n, slot, stream). */
#define STREAM_EVENT 0u /* slot 0: pair 0 = waiting time, pair 1 = reaction pick */
#define STREAM_FIRST 1u /* slot j/2: pair (j mod 2) = inversion uniform of j    */
#define STREAM_PTRS 2u  /* slot j, stream 2+r: PTRS iteration r of reaction j   */

#define INV_KMAX 100        /* inversion search cap (tail below 2^-53 for lam < 10) */
#define PTRS_RMAX 1000u     /* PTRS iteration cap (acceptance is ~0.9 per round)    */
#define K_CLAMP 2147483648.0 /* 2^31: larger draws are clamped (state cannot hold them) */

static void block(uint64_t seed, uint32_t traj, uint32_t n, uint32_t slot, uint32_t stream,
                  uint32_t w[4]) {
  uint32_t ctr[4] = {traj, n, slot, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* Poisson(lam).  lam < 10: sequential search of the CDF from k = 0 with one
 * uniform, p_k = p_{k-1} * (lam * (1/k)).  lam >= 10: Hoermann's transformed
 * rejection with squeeze (PTRS), each round taking its own (U, V) pair. */
int64_t orc_poisson(double lam, uint64_t seed, uint32_t traj, uint32_t n, int32_t j,
                    orc_ops *ops) {
  uint32_t w[4];
  if (!(lam > 0.0)) return 0;
  if (lam < 10.0) {
    block(seed, traj, n, (uint32_t)j >> 1, STREAM_FIRST, w);
    int p = j & 1;
    double u = orc_u53(w[2 * p], w[2 * p + 1]);
    double pk = exp(-lam);
    double F = pk;
    int64_t k = 0;
    if (ops) ops->inv_draws++;
    while (u > F && k < INV_KMAX) {
      k = k + 1;
      pk = pk * (lam * (1.0 / (double)k));
      F = F + pk;
      if (ops) ops->inv_iters++;
    }
    return k;
  }
  if (ops) ops->ptrs_draws++;
  double smu = sqrt(lam);
  double b = 0.931 + 2.53 * smu;
  double a = -0.059 + 0.02483 * b;
  double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  double vr = 0.9277 - 3.6224 / (b - 2.0);
  double loglam = log(lam);
  for (uint32_t r = 0; r < PTRS_RMAX; ++r) {
    block(seed, traj, n, (uint32_t)j, STREAM_PTRS + r, w);
    if (ops) { ops->ptrs_iters++; ops->philox_blocks++; }
    double U = orc_u53(w[0], w[1]) - 0.5;
    double V = orc_u53(w[2], w[3]);
    double us = 0.5 - fabs(U);
    double kf = floor((2.0 * a / us + b) * U + lam + 0.43);
    if (us >= 0.07 && V <= vr) return (int64_t)(kf < K_CLAMP ? kf : K_CLAMP);
    if (kf < 0.0 || (us < 0.013 && V > us)) continue;
    if (ops) ops->ptrs_log_tests++;
    double lhs = log(V * inv_alpha / (a / (us * us) + b));
    double rhs = -lam + kf * loglam - lgamma(kf + 1.0);
    if (lhs <= rhs) return (int64_t)(kf < K_CLAMP ? kf : K_CLAMP);
  }
  {
    double kf = floor(lam);
    return (int64_t)(kf < K_CLAMP ? kf : K_CLAMP);
  }
}

/* Chemical Langevin increment (the CLE-based approximation of the paper's
 * Methods section, applied to one reaction's firings over a leap): the Poisson
 * count is replaced by a Gaussian of the same mean and variance, rounded to the
 * nearest integer and floored at zero.  z = sqrt(-2 ln(1-u1)) cos(2 pi u2)
 * (Box-Muller), (u1, u2) from the reaction's first PTRS block. */
int64_t orc_cle_count(double lam, uint64_t seed, uint32_t traj, uint32_t n, int32_t j) {
  uint32_t w[4];
  block(seed, traj, n, (uint32_t)j, STREAM_PTRS, w);
  double u1 = orc_u53(w[0], w[1]);
  double u2 = orc_u53(w[2], w[3]);
  double z = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
  double kf = floor(lam + sqrt(lam) * z + 0.5);
  if (kf < 0.0) kf = 0.0;
  return (int64_t)(kf < K_CLAMP ? kf : K_CLAMP);
}

void orc_cle_many(double lam, uint64_t seed, uint32_t n0, int32_t j, int64_t n, int64_t *out) {
  for (int64_t t = 0; t < n; ++t) out[t] = orc_cle_count(lam, seed, (uint32_t)t, n0, j);
}

/* ------------------------------------------------------------------------- */
/* Network preprocessing                                                     */
/* ------------------------------------------------------------------------- */

typedef struct {
  int N, M;
  int *kind;   /* 0 source, 1 first order, 2 two distinct species, 3 homodimer */
  int *ra, *rb;
  int *nu;     /* dense net change nu[j*N + i] = products - reactants        */
  int *hor;    /* highest order of a reaction consuming species i as reactant */
  int *dimer;  /* some reaction takes two molecules of species i             */
} onet;

static void onet_free(onet *g) {
  free(g->kind); free(g->ra); free(g->rb); free(g->nu); free(g->hor); free(g->dimer);
}

static int onet_build(const orc_net_desc *d, onet *g) {
  memset(g, 0, sizeof(*g));
  if (!d || d->n_species <= 0 || d->n_reactions <= 0) return ORC_E_ARG;
  int N = d->n_species, M = d->n_reactions;
  g->N = N; g->M = M;
  g->kind = calloc(M, sizeof(int)); g->ra = calloc(M, sizeof(int)); g->rb = calloc(M, sizeof(int));
  g->nu = calloc((size_t)M * N, sizeof(int));
  g->hor = calloc(N, sizeof(int)); g->dimer = calloc(N, sizeof(int));
  int *rc = calloc(N, sizeof(int));
  if (!g->kind || !g->ra || !g->rb || !g->nu || !g->hor || !g->dimer || !rc) {
    free(rc); onet_free(g); return ORC_E_NOMEM;
  }
  int err = ORC_OK;
  for (int j = 0; j < M && !err; ++j) {
    memset(rc, 0, N * sizeof(int));
    int order = 0;
    for (int e = d->react_ptr[j]; e < d->react_ptr[j + 1]; ++e) {
      int s = d->react_species[e], c = d->react_coeff[e];
      if (s < 0 || s >= N || c <= 0 || c > (1 << 20)) { err = ORC_E_NET; break; }
      rc[s] += c; order += c;
      if (order > 2) { err = ORC_E_ORDER; break; }
    }
    if (err) break;
    for (int e = d->prod_ptr[j]; e < d->prod_ptr[j + 1]; ++e) {
      int s = d->prod_species[e], c = d->prod_coeff[e];
      if (s < 0 || s >= N || c <= 0 || c > (1 << 20)) { err = ORC_E_NET; break; }
      g->nu[(size_t)j * N + s] += c;
    }
    if (err) break;
    int first = -1, second = -1;
    for (int i = 0; i < N; ++i) {
      if (rc[i] == 0) continue;
      g->nu[(size_t)j * N + i] -= rc[i];
      if (first < 0) first = i; else second = i;
      if (order > g->hor[i]) g->hor[i] = order;
      if (rc[i] == 2) g->dimer[i] = 1;
    }
    if (order == 0) g->kind[j] = 0;
    else if (order == 1) { g->kind[j] = 1; g->ra[j] = first; }
    else if (second >= 0) { g->kind[j] = 2; g->ra[j] = first; g->rb[j] = second; }
    else { g->kind[j] = 3; g->ra[j] = first; }
  }
  free(rc);
  if (err) onet_free(g);
  return err;
}

/* ------------------------------------------------------------------------- */
/* One trajectory                                                            */
/* ------------------------------------------------------------------------- */

/* Mass-action propensity a_j = c_j * h_j(x): h = 1, x_a, x_a*x_b or
 * x_a*(x_a-1)/2 (number of distinct reactant combinations). */
static double propensity(const onet *g, int j, double c, const int32_t *x) {
  double h;
  switch (g->kind[j]) {
    case 0: h = 1.0; break;
    case 1: h = (double)x[g->ra[j]]; break;
    case 2: h = (double)x[g->ra[j]] * (double)x[g->rb[j]]; break;
    default: { double xa = (double)x[g->ra[j]]; h = 0.5 * (xa * (xa - 1.0)); } break;
  }
  return c * h;
}

typedef struct {
  const onet *g;
  const orc_params *par;
  const double *c; int64_t c_ld;
  const double *times; int S;
  uint32_t traj;
  int32_t *out; int64_t out_ld;
  int32_t *x; int64_t *xn; double *a; int *crit; int64_t *k;
  double t; uint32_t n; int s;
  uint64_t leaps, ssa, rej, status;
  orc_ops *ops;
} traj_state;

static void record(traj_state *T, int s) {
  for (int i = 0; i < T->g->N; ++i) T->out[((int64_t)s * T->g->N + i) * T->out_ld] = T->x[i];
}

/* Samples at or before t take the current state. Returns 1 when all are taken. */
static int record_through(traj_state *T) {
  while (T->s < T->S && T->times[T->s] <= T->t) record(T, T->s++);
  return T->s == T->S;
}

static void fill_rest(traj_state *T) {
  while (T->s < T->S) record(T, T->s++);
}

static double all_propensities(traj_state *T) {
  const onet *g = T->g;
  double a0 = 0.0;
  for (int j = 0; j < g->M; ++j) {
    T->a[j] = propensity(g, j, T->c[(int64_t)j * T->c_ld], T->x);
    a0 = a0 + T->a[j];
  }
  if (T->ops) T->ops->prop_evals += g->M;
  return a0;
}

static uint64_t steps_taken(const traj_state *T) { return T->leaps + T->ssa + T->rej; }

/* The direct method's selection (Gillespie 1977): the first j, in index order
 * among the allowed ones, whose running sum a_0 + ... + a_j exceeds r; when
 * rounding leaves none, the last allowed j with a_j > 0.  *terms counts the
 * terms added. */
static int pick_index(const double *a, int m, double r, const int *allowed, uint64_t *terms) {
  double acc = 0.0;
  int last = -1;
  for (int j = 0; j < m; ++j) {
    if (allowed && !allowed[j]) continue;
    if (terms) ++*terms;
    acc = acc + a[j];
    if (a[j] > 0.0) last = j;
    if (r < acc) return j;
  }
  return last;
}

static int pick_reaction(traj_state *T, double r, const int *allowed) {
  return pick_index(T->a, T->g->M, r, allowed, T->ops ? &T->ops->select_terms : NULL);
}

/* The critical race of Cao, Gillespie and Petzold (2006): a critical reaction
 * fires when its waiting time tau'' is no longer than the leap bound tau'; here
 * also no later than the next sample time (delta away). */
static int critical_fires(double tau_c, double tau_p, double delta) {
  return (tau_c <= tau_p) && (tau_c <= delta);
}

int orc_pick_index(const double *a, int m, double r, const int *allowed) {
  return pick_index(a, m, r, allowed, NULL);
}

int orc_critical_fires(double tau_c, double tau_p, double delta) {
  return critical_fires(tau_c, tau_p, delta);
}

/* Result codes of the exact-event loop. */
#define BURST_CONTINUE 0
#define BURST_DONE 1

/* Up to `count` exact SSA events (count < 0: until the end).  Each event draws
 * its waiting time Exp(a0) and picks reaction j with probability a_j / a0.
 * Samples strictly before the event time take the pre-event state; a sample
 * at exactly the event time takes the post-event state. */
static int ssa_events(traj_state *T, int64_t count) {
  const onet *g = T->g;
  for (int64_t e = 0; count < 0 || e < count; ++e) {
    if (steps_taken(T) >= T->par->max_steps) { T->status |= ORC_ST_MAXSTEPS; fill_rest(T); return BURST_DONE; }
    double a0 = all_propensities(T);
    if (a0 == 0.0) { T->status |= ORC_ST_ABSORBED; fill_rest(T); return BURST_DONE; }
    uint32_t w[4];
    block(T->par->seed, T->traj, T->n, 0u, STREAM_EVENT, w);
    if (T->ops) { T->ops->philox_blocks++; T->ops->exp_draws++; }
    double u1 = orc_u53(w[0], w[1]);
    double u2 = orc_u53(w[2], w[3]);
    double tau = -log(1.0 - u1) / a0;
    double tn = T->t + tau;
    while (T->s < T->S && T->times[T->s] < tn) record(T, T->s++);
    if (T->s == T->S) return BURST_DONE;
    int j = pick_reaction(T, u2 * a0, NULL);
    if (j < 0) { T->status |= ORC_ST_ABSORBED; fill_rest(T); return BURST_DONE; }
    int ovf = 0;
    for (int i = 0; i < g->N; ++i) {
      int v = g->nu[(size_t)j * g->N + i];
      if (!v) continue;
      int64_t y = (int64_t)T->x[i] + v;
      if (y > INT32_MAX || y < 0) ovf = 1;
      if (T->ops) T->ops->update_terms++;
    }
    if (ovf) { T->status |= ORC_ST_OVERFLOW; fill_rest(T); return BURST_DONE; }
    for (int i = 0; i < g->N; ++i) T->x[i] += g->nu[(size_t)j * g->N + i];
    T->t = tn;
    T->n++;
    T->ssa++;
    if (record_through(T)) return BURST_DONE;
  }
  return BURST_CONTINUE;
}

static void simulate(traj_state *T) {
  const onet *g = T->g;
  const orc_params *P = T->par;
  const int N = g->N, M = g->M;
  T->t = 0.0; T->n = 0; T->s = 0;
  T->leaps = T->ssa = T->rej = T->status = 0;
  if (record_through(T)) return;
  if (P->method == 1) { ssa_events(T, -1); return; }
  for (;;) {
    /* Propensities and total rate. */
    if (steps_taken(T) >= P->max_steps) { T->status |= ORC_ST_MAXSTEPS; fill_rest(T); return; }
    double a0 = all_propensities(T);
    if (a0 == 0.0) { T->status |= ORC_ST_ABSORBED; fill_rest(T); return; }

    /* Critical reactions: a_j > 0 and fewer than n_c firings would exhaust a
     * consumed reactant, L_j = min over consumed i of floor(x_i / |nu_ij|). */
    for (int j = 0; j < M; ++j) {
      int64_t L = -1;
      for (int i = 0; i < N; ++i) {
        int v = g->nu[(size_t)j * N + i];
        if (v >= 0) continue;
        int64_t l = (int64_t)T->x[i] / (int64_t)(-v);
        if (L < 0 || l < L) L = l;
        if (T->ops) T->ops->crit_tests++;
      }
      T->crit[j] = (T->a[j] > 0.0) && (L >= 0) && (L < P->n_c);
    }

    /* Leap size from the species-based bound: for every reactant species i,
     * mu_i and sigma^2_i summed over the non-critical reactions, then
     * tau' = min_i min(b_i/|mu_i|, b_i^2/sigma^2_i), b_i = max(eps*x_i/g_i, 1). */
    double tau_p = INFINITY;
    for (int i = 0; i < N; ++i) {
      if (g->hor[i] == 0) continue;
      double mu = 0.0, sig = 0.0;
      for (int j = 0; j < M; ++j) {
        int v = g->nu[(size_t)j * N + i];
        if (v == 0 || T->crit[j]) continue;
        mu = mu + (double)v * T->a[j];
        sig = sig + (double)(v * v) * T->a[j];
        if (T->ops) T->ops->tau_terms++;
      }
      if (T->ops) T->ops->tau_species++;
      int32_t xi = T->x[i];
      double bnd = 1.0;
      if (xi > 1) {
        double gi = 1.0;
        if (g->hor[i] == 2) gi = g->dimer[i] ? 2.0 + 1.0 / (double)(xi - 1) : 2.0;
        bnd = P->eps * (double)xi / gi;
        if (bnd < 1.0) bnd = 1.0;
      }
      if (mu != 0.0) { double q = bnd / fabs(mu); if (q < tau_p) tau_p = q; }
      if (sig != 0.0) { double q = (bnd * bnd) / sig; if (q < tau_p) tau_p = q; }
    }

    for (;;) {
      if (steps_taken(T) >= P->max_steps) { T->status |= ORC_ST_MAXSTEPS; fill_rest(T); return; }
      /* Too short a leap: take a burst of exact events instead. */
      if (tau_p < P->ssa_factor / a0) {
        if (ssa_events(T, P->ssa_burst) == BURST_DONE) return;
        break;
      }
      /* Critical race: the first critical firing is Exp(a0c); it wins when it
       * comes no later than both tau' and the next sample time. */
      double a0c = 0.0;
      for (int j = 0; j < M; ++j) if (T->crit[j]) a0c = a0c + T->a[j];
      uint32_t ev[4] = {0, 0, 0, 0};
      double tau_c = INFINITY;
      if (a0c > 0.0) {
        block(P->seed, T->traj, T->n, 0u, STREAM_EVENT, ev);
        if (T->ops) { T->ops->philox_blocks++; T->ops->exp_draws++; }
        tau_c = -log(1.0 - orc_u53(ev[0], ev[1])) / a0c;
      }
      double delta = T->times[T->s] - T->t;
      int fire = critical_fires(tau_c, tau_p, delta);
      double tau = fire ? tau_c : (tau_p < delta ? tau_p : delta);

      /* Poisson firings of every non-critical reaction over tau; one firing of
       * one critical reaction when the race was won. */
      int last_pair = -1;
      for (int j = 0; j < M; ++j) {
        T->k[j] = 0;
        if (T->crit[j]) continue;
        double lam = T->a[j] * tau;
        if (lam > 0.0 && lam < 10.0 && (j >> 1) != last_pair) {
          last_pair = j >> 1;
          if (T->ops) T->ops->philox_blocks++;
        }
        if (P->cle_threshold > 0.0 && lam >= P->cle_threshold)
          T->k[j] = orc_cle_count(lam, P->seed, T->traj, T->n, j);
        else
          T->k[j] = orc_poisson(lam, P->seed, T->traj, T->n, j, T->ops);
      }
      if (fire) {
        int jc = pick_reaction(T, orc_u53(ev[2], ev[3]) * a0c, T->crit);
        if (jc < 0) { T->status |= ORC_ST_ABSORBED; fill_rest(T); return; }
        T->k[jc] = 1;
      }

      /* Candidate state, exactly in 64-bit integers. */
      for (int i = 0; i < N; ++i) T->xn[i] = T->x[i];
      for (int j = 0; j < M; ++j) {
        if (T->k[j] == 0) continue;
        for (int i = 0; i < N; ++i) {
          int v = g->nu[(size_t)j * N + i];
          if (!v) continue;
          T->xn[i] += T->k[j] * (int64_t)v;
          if (T->ops) T->ops->update_terms++;
        }
      }
      int neg = 0, big = 0;
      for (int i = 0; i < N; ++i) {
        if (T->xn[i] < 0) neg = 1;
        else if (T->xn[i] > INT32_MAX) big = 1;
      }
      if (neg) {
        /* A count would go negative: halve tau' and try again with fresh draws. */
        tau_p = tau_p * 0.5;
        T->n++;
        T->rej++;
        continue;
      }
      if (big) { T->status |= ORC_ST_OVERFLOW; fill_rest(T); return; }
      for (int i = 0; i < N; ++i) T->x[i] = (int32_t)T->xn[i];
      if (tau == delta) T->t = T->times[T->s];
      else T->t = T->t + tau;
      T->n++;
      T->leaps++;
      if (record_through(T)) return;
      break;
    }
  }
}

int orc_run(const orc_net_desc *net, const double *rates, int64_t rates_ld,
            const int32_t *x0, int64_t x0_ld, const double *times, int32_t n_times,
            int64_t traj_first, int64_t n_traj, int32_t *out, int64_t out_ld,
            uint64_t *stats, const orc_params *par, orc_ops *ops) {
  if (!net || !rates || !x0 || !times || !out || !stats || !par) return ORC_E_ARG;
  if (n_times <= 0 || n_traj < 0 || traj_first < 0 || traj_first + n_traj > 4294967296LL)
    return ORC_E_ARG;
  if (par->ssa_burst < 1 || par->max_steps < 1 || !(par->eps > 0.0) || !(par->ssa_factor >= 0.0))
    return ORC_E_ARG;
  if (!(par->cle_threshold == 0.0 || par->cle_threshold >= 10.0)) return ORC_E_ARG;
  for (int s = 0; s < n_times; ++s) {
    if (!(times[s] >= 0.0) || !isfinite(times[s])) return ORC_E_ARG;
    if (s > 0 && !(times[s] > times[s - 1])) return ORC_E_ARG;
  }
  onet g;
  int err = onet_build(net, &g);
  if (err) return err;
  int N = g.N, M = g.M;
  traj_state T;
  memset(&T, 0, sizeof(T));
  T.x = malloc(N * sizeof(int32_t));
  T.xn = malloc(N * sizeof(int64_t));
  T.a = malloc(M * sizeof(double));
  T.crit = malloc(M * sizeof(int));
  T.k = malloc(M * sizeof(int64_t));
  if (!T.x || !T.xn || !T.a || !T.crit || !T.k) {
    free(T.x); free(T.xn); free(T.a); free(T.crit); free(T.k); onet_free(&g);
    return ORC_E_NOMEM;
  }
  T.g = &g; T.par = par; T.times = times; T.S = n_times; T.ops = ops; T.out_ld = out_ld;
  for (int64_t t = 0; t < n_traj; ++t) {
    T.c = rates + t; T.c_ld = rates_ld;
    T.traj = (uint32_t)(traj_first + t);
    T.out = out + t;
    for (int i = 0; i < N; ++i) T.x[i] = x0_ld ? x0[(int64_t)i * x0_ld + t] : x0[i];
    simulate(&T);
    stats[t * 4 + 0] = T.leaps;
    stats[t * 4 + 1] = T.ssa;
    stats[t * 4 + 2] = T.rej;
    stats[t * 4 + 3] = T.status;
    if (ops) { ops->leaps += T.leaps; ops->ssa_events += T.ssa; ops->rejections += T.rej; }
  }
  free(T.x); free(T.xn); free(T.a); free(T.crit); free(T.k);
  onet_free(&g);
  return ORC_OK;
}

/* n Poisson(lam) variates for reaction slot j of attempt n0, trajectory ids
 * 0..n-1 (a test helper: distinct trajectory ids give independent streams). */
void orc_poisson_many(double lam, uint64_t seed, uint32_t n0, int32_t j, int64_t n, int64_t *out) {
  for (int64_t t = 0; t < n; ++t) out[t] = orc_poisson(lam, seed, (uint32_t)t, n0, j, NULL);
}
