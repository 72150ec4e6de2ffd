/*
 * ode.c -- plain FP64 CPU oracle for the deterministic reaction-rate-equation
 * sweep.  TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline).
 *
 * Model (paper, Methods section): for abundant species the counts follow the
 * reaction-rate equations dy/dt = sum_j nu_j a_j(y) with continuous mass-action
 * rates a_j = c_j * h_j(y), h_j = 1, y_a, y_a*y_b, or y_a^2/2 for a homodimer
 * (the large-number limit of c*x(x-1)/2).
 *
 * Integrator: the Dormand-Prince 5(4) pair (J. R. Dormand, P. J. Prince,
 * J. Comput. Appl. Math. 6 (1980) 19) with first-same-as-last stages; the
 * fifth-order solution is propagated and the embedded fourth-order one gives
 * the error estimate.  Error norm: root mean square over species of
 * e_i / (atol + rtol * max(|y_i|, |y_new_i|)).  A step is accepted when the
 * norm is <= 1; the next step is h * min(5, max(0.2, 0.9 * err^(-1/5))) (after
 * a rejection the growth factor is capped at 1).  The first step is
 * 0.01 * rms(y/sc) / rms(f/sc) (1e-6 when either norm is below 1e-5).  A step
 * that reaches the next sample time ends exactly on it.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef struct {
  int N, M;
  int *kind, *ra, *rb; /* 0 source, 1 first order, 2 pair, 3 homodimer */
  int *nu;             /* dense nu[j*N + i] */
} dnet;

static void dnet_free(dnet *g) { free(g->kind); free(g->ra); free(g->rb); free(g->nu); }

static int dnet_build(const orc_net_desc *d, dnet *g) {
  memset(g, 0, sizeof(*g));
  if (!d || d->n_species <= 0 || d->n_reactions <= 0) return ORC_E_ARG;
  int N = d->n_species, M = d->n_reactions;
  g->N = N; g->M = M;
  g->kind = calloc(M, sizeof(int)); g->ra = calloc(M, sizeof(int)); g->rb = calloc(M, sizeof(int));
  g->nu = calloc((size_t)M * N, sizeof(int));
  int *rc = calloc(N, sizeof(int));
  if (!g->kind || !g->ra || !g->rb || !g->nu || !rc) { free(rc); dnet_free(g); return ORC_E_NOMEM; }
  for (int j = 0; j < M; ++j) {
    memset(rc, 0, N * sizeof(int));
    int order = 0;
    for (int e = d->react_ptr[j]; e < d->react_ptr[j + 1]; ++e) {
      int s = d->react_species[e], c = d->react_coeff[e];
      if (s < 0 || s >= N || c <= 0 || c > (1 << 20)) { free(rc); dnet_free(g); return ORC_E_NET; }
      rc[s] += c; order += c;
      if (order > 2) { free(rc); dnet_free(g); return ORC_E_ORDER; }
    }
    for (int e = d->prod_ptr[j]; e < d->prod_ptr[j + 1]; ++e) {
      int s = d->prod_species[e], c = d->prod_coeff[e];
      if (s < 0 || s >= N || c <= 0 || c > (1 << 20)) { free(rc); dnet_free(g); return ORC_E_NET; }
      g->nu[(size_t)j * N + s] += c;
    }
    int first = -1, second = -1;
    for (int i = 0; i < N; ++i) {
      if (!rc[i]) continue;
      g->nu[(size_t)j * N + i] -= rc[i];
      if (first < 0) first = i; else second = i;
    }
    if (order == 0) g->kind[j] = 0;
    else if (order == 1) { g->kind[j] = 1; g->ra[j] = first; }
    else if (second >= 0) { g->kind[j] = 2; g->ra[j] = first; g->rb[j] = second; }
    else { g->kind[j] = 3; g->ra[j] = first; }
  }
  free(rc);
  return ORC_OK;
}

/* f = dy/dt at y; reactions in index order, each adding nu_ij * a_j. */
static void rhs(const dnet *g, const double *c, int64_t cld, const double *y, double *f) {
  for (int i = 0; i < g->N; ++i) f[i] = 0.0;
  for (int j = 0; j < g->M; ++j) {
    double h;
    switch (g->kind[j]) {
      case 0: h = 1.0; break;
      case 1: h = y[g->ra[j]]; break;
      case 2: h = y[g->ra[j]] * y[g->rb[j]]; break;
      default: h = 0.5 * (y[g->ra[j]] * y[g->ra[j]]); break;
    }
    double a = c[(int64_t)j * cld] * h;
    for (int i = 0; i < g->N; ++i) {
      int v = g->nu[(size_t)j * g->N + i];
      if (v) f[i] = f[i] + (double)v * a;
    }
  }
}

/* Dormand-Prince 5(4) tableau (the system is autonomous, so the stage times
 * are not needed). */
static const double A21 = 1.0 / 5.0;
static const double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
static const double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
static const double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
                    A54 = -212.0 / 729.0;
static const double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0,
                    A64 = 49.0 / 176.0, A65 = -5103.0 / 18656.0;
static const double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0,
                    B5 = -2187.0 / 6784.0, B6 = 11.0 / 84.0;
static const double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0,
                    E5 = -17253.0 / 339200.0, E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;

int orc_ode_run(const orc_net_desc *net, const double *rates, int64_t rates_ld,
                const int32_t *x0, int64_t x0_ld, const double *times, int32_t n_times,
                int64_t n_traj, double *out, int64_t out_ld, uint64_t *stats,
                const orc_ode_params *par) {
  if (!net || !rates || !x0 || !times || !out || !stats || !par) return ORC_E_ARG;
  if (n_times <= 0 || n_traj < 0 || !(par->rtol > 0.0) || !(par->atol > 0.0) || par->max_steps < 1)
    return ORC_E_ARG;
  for (int s = 0; s < n_times; ++s) {
    if (!(times[s] >= 0.0) || !isfinite(times[s])) return ORC_E_ARG;
    if (s > 0 && !(times[s] > times[s - 1])) return ORC_E_ARG;
  }
  dnet g;
  int err = dnet_build(net, &g);
  if (err) return err;
  const int N = g.N;
  double *w = malloc(sizeof(double) * (size_t)N * 10);
  if (!w) { dnet_free(&g); return ORC_E_NOMEM; }
  double *y = w, *yn = w + N, *k1 = w + 2 * N, *k2 = w + 3 * N, *k3 = w + 4 * N, *k4 = w + 5 * N,
         *k5 = w + 6 * N, *k6 = w + 7 * N, *k7 = w + 8 * N, *ys = w + 9 * N;
  for (int64_t t = 0; t < n_traj; ++t) {
    const double *c = rates + t;
    for (int i = 0; i < N; ++i) y[i] = (double)(x0_ld ? x0[(int64_t)i * x0_ld + t] : x0[i]);
    double tt = 0.0;
    int s = 0;
    uint64_t acc = 0, rej = 0, status = 0;
    while (s < n_times && times[s] <= tt) {
      for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
      s++;
    }
    rhs(&g, c, rates_ld, y, k1);
    /* first step */
    double d0 = 0.0, d1 = 0.0;
    for (int i = 0; i < N; ++i) {
      double sc = par->atol + par->rtol * fabs(y[i]);
      d0 = d0 + (y[i] / sc) * (y[i] / sc);
      d1 = d1 + (k1[i] / sc) * (k1[i] / sc);
    }
    d0 = sqrt(d0 / N);
    d1 = sqrt(d1 / N);
    double h = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
    int last_rejected = 0;
    while (s < n_times) {
      if (acc + rej >= par->max_steps) { status |= ORC_ST_MAXSTEPS; break; }
      double delta = times[s] - tt;
      int clip = !(h < delta);
      double hu = clip ? delta : h;
      for (int i = 0; i < N; ++i) ys[i] = y[i] + hu * (A21 * k1[i]);
      rhs(&g, c, rates_ld, ys, k2);
      for (int i = 0; i < N; ++i) ys[i] = y[i] + hu * (A31 * k1[i] + A32 * k2[i]);
      rhs(&g, c, rates_ld, ys, k3);
      for (int i = 0; i < N; ++i) ys[i] = y[i] + hu * (A41 * k1[i] + A42 * k2[i] + A43 * k3[i]);
      rhs(&g, c, rates_ld, ys, k4);
      for (int i = 0; i < N; ++i)
        ys[i] = y[i] + hu * (A51 * k1[i] + A52 * k2[i] + A53 * k3[i] + A54 * k4[i]);
      rhs(&g, c, rates_ld, ys, k5);
      for (int i = 0; i < N; ++i)
        ys[i] = y[i] + hu * (A61 * k1[i] + A62 * k2[i] + A63 * k3[i] + A64 * k4[i] + A65 * k5[i]);
      rhs(&g, c, rates_ld, ys, k6);
      for (int i = 0; i < N; ++i)
        yn[i] = y[i] + hu * (B1 * k1[i] + B3 * k3[i] + B4 * k4[i] + B5 * k5[i] + B6 * k6[i]);
      rhs(&g, c, rates_ld, yn, k7);
      double e2 = 0.0;
      for (int i = 0; i < N; ++i) {
        double e = hu * (E1 * k1[i] + E3 * k3[i] + E4 * k4[i] + E5 * k5[i] + E6 * k6[i] + E7 * k7[i]);
        double ay = fabs(y[i]), an = fabs(yn[i]);
        double sc = par->atol + par->rtol * (ay > an ? ay : an);
        e2 = e2 + (e / sc) * (e / sc);
      }
      double en = sqrt(e2 / N);
      if (en <= 1.0) {
        double fac = en == 0.0 ? 5.0 : 0.9 * pow(en, -0.2);
        if (fac > 5.0) fac = 5.0;
        if (fac < 0.2) fac = 0.2;
        if (last_rejected && fac > 1.0) fac = 1.0;
        memcpy(y, yn, sizeof(double) * N);
        memcpy(k1, k7, sizeof(double) * N);
        if (clip) tt = times[s];
        else tt = tt + hu;
        h = hu * fac;
        acc++;
        last_rejected = 0;
        while (s < n_times && times[s] <= tt) {
          for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
          s++;
        }
      } else {
        double fac = 0.9 * pow(en, -0.2);
        if (fac < 0.2) fac = 0.2;
        h = hu * fac;
        rej++;
        last_rejected = 1;
      }
    }
    while (s < n_times) {
      for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
      s++;
    }
    stats[t * 4 + 0] = acc;
    stats[t * 4 + 1] = rej;
    stats[t * 4 + 2] = 0;
    stats[t * 4 + 3] = status;
  }
  free(w);
  dnet_free(&g);
  return ORC_OK;
}
