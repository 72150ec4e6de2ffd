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
 *
 * Stiff integrator (method ORC_ODE_ROS4): a linearly implicit Rosenbrock
 * method of order 4 with an embedded order-3 solution, the gamma = 1/2
 * parameter set of L. F. Shampine, ACM Trans. Math. Softw. 8 (1982) 93, in the
 * transformed form of Hairer and Wanner (Solving ODEs II, Sec. IV.7), where no
 * product of the Jacobian with a vector is needed.  With J the exact Jacobian
 * of the rate equations at y and W = (1/(gamma h)) I - J, each step solves
 *   W u1 = f(y)
 *   W u2 = f(y + a21 u1)            + (c21 u1) / h
 *   W u3 = f(y + a31 u1 + a32 u2)   + (c31 u1 + c32 u2) / h
 *   W u4 = f(y + a31 u1 + a32 u2)   + (c41 u1 + c42 u2 + c43 u3) / h
 * (the fourth stage reuses the third stage's argument) and takes
 * y' = y + sum m_i u_i, with the error estimate sum e_i u_i (the difference
 * from the order-3 solution).  W is factored once per step by Gaussian
 * elimination with partial pivoting.  The error norm and the step rules are
 * those above with the exponent -1/4 of an order-3 error estimate.
 *
 * Hybrid stochastic/deterministic sweep (paper, Methods section: abundant
 * species follow the mean-field equations while low-amount species keep their
 * random fluctuations; the process is a piecewise-deterministic Markov process,
 * M. H. A. Davis, J. R. Stat. Soc. B 46 (1984) 353).  The caller partitions the
 * reactions: continuous ones drive the flow dy/dt = sum_{j in C} nu_j a_j(y)
 * (the rates above), discrete ones fire as jumps y += nu_j with intensities
 * a_j = max(0, c_j * h_j(y)), h_j = 1, y_a, y_a*y_b or y_a*(y_a-1)/2 (the
 * stochastic mass-action forms).  Jump times follow the integrated-intensity
 * construction of hybrid methods such as Salis and Kaznessis (J. Chem. Phys.
 * 122, 054103 (2005)): with xi ~ Exp(1), the next jump comes when
 * L(t) = integral of a0_D(y) since the last jump reaches xi.  L is integrated
 * with y by the same Dormand-Prince step (its own error term enters the norm as
 * max(rms over species, |e_L| / sc_L)); when an accepted step carries L past
 * xi, its length is searched from the same start by the Illinois variant of
 * regula falsi (M. Dowell, P. Jarratt, BIT 11 (1971) 168) on g = L - xi until
 * |g| <= 1e-12 (1 + xi) or 30 trials, and the jump fires at the end of the last
 * trial.  The jumping reaction is the first discrete j
 * with u * a0_D < a_1 + ... + a_j at that state.  Jump k of trajectory tr draws
 * (xi, u) from Philox4x32-10 block (tr, k, 0, 0x80000000): xi = -log(1 - u53(w0,
 * w1)), u = u53(w2, w3).
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

/* Rosenbrock 4(3) coefficients, transformed form (Shampine 1982, gamma = 1/2). */
static const double RG = 0.5;
static const double RA21 = 2.0, RA31 = 48.0 / 25.0, RA32 = 6.0 / 25.0;
static const double RC21 = -8.0, RC31 = 372.0 / 25.0, RC32 = 12.0 / 5.0;
static const double RC41 = -112.0 / 125.0, RC42 = -54.0 / 125.0, RC43 = -2.0 / 5.0;
static const double RM1 = 19.0 / 9.0, RM2 = 1.0 / 2.0, RM3 = 25.0 / 108.0, RM4 = 125.0 / 108.0;
static const double RE1 = 17.0 / 54.0, RE2 = 7.0 / 36.0, RE3 = 0.0, RE4 = 125.0 / 108.0;

/* Exact Jacobian of the rate equations at y, dense row-major jac[i*N + k]:
 * every reaction j in increasing index adds nu_ij * d a_j / d y_k to row i,
 * with d(c y_a)/dy_a = c, d(c y_a y_b)/dy_a = c y_b, d(c y_a y_b)/dy_b = c y_a
 * and d(c y_a^2 / 2)/dy_a = c y_a. */
static void jacobian(const dnet *g, const double *c, int64_t cld, const double *y, double *jac) {
  const int N = g->N;
  for (int e = 0; e < N * N; ++e) jac[e] = 0.0;
  for (int j = 0; j < g->M; ++j) {
    const double cj = c[(int64_t)j * cld];
    int ka = -1, kb = -1;
    double da = 0.0, db = 0.0;
    switch (g->kind[j]) {
      case 0: break;
      case 1: ka = g->ra[j]; da = cj; break;
      case 2: ka = g->ra[j]; da = cj * y[g->rb[j]]; kb = g->rb[j]; db = cj * y[g->ra[j]]; break;
      default: ka = g->ra[j]; da = cj * y[g->ra[j]]; break;
    }
    for (int i = 0; i < N; ++i) {
      const int v = g->nu[(size_t)j * N + i];
      if (!v) continue;
      if (ka >= 0) jac[i * N + ka] = jac[i * N + ka] + (double)v * da;
      if (kb >= 0) jac[i * N + kb] = jac[i * N + kb] + (double)v * db;
    }
  }
}

/* In-place LU factorization with partial pivoting: the pivot of column k is
 * the first row r >= k of largest |a[r][k]|, rows k and r are exchanged (perm
 * records it), multipliers l = a[i][k] / a[k][k] are stored below the diagonal
 * and each a[i][j] (j > k) becomes a[i][j] - l * a[k][j].  A zero pivot is not
 * an error: the solve then yields infinities or NaNs, which the step controller
 * rejects. */
static void lu_factor(int N, double *a, int *perm) {
  for (int k = 0; k < N; ++k) {
    int r = k;
    double best = fabs(a[k * N + k]);
    for (int i = k + 1; i < N; ++i) {
      const double v = fabs(a[i * N + k]);
      if (v > best) { best = v; r = i; }
    }
    perm[k] = r;
    if (r != k) {
      for (int j = 0; j < N; ++j) {
        const double tmp = a[k * N + j];
        a[k * N + j] = a[r * N + j];
        a[r * N + j] = tmp;
      }
    }
    for (int i = k + 1; i < N; ++i) {
      const double l = a[i * N + k] / a[k * N + k];
      a[i * N + k] = l;
      for (int j = k + 1; j < N; ++j) a[i * N + j] = a[i * N + j] - l * a[k * N + j];
    }
  }
}

/* Solve (LU) x = P b in place on b: the row exchanges in factorization order,
 * forward substitution with unit L (each x_i subtracts l_ik x_k for k in
 * increasing order), then back substitution (each x_i subtracts u_ik x_k for
 * k in decreasing order, then divides by u_ii). */
static void lu_solve(int N, const double *a, const int *perm, double *b) {
  for (int k = 0; k < N; ++k) {
    const int r = perm[k];
    if (r != k) { const double tmp = b[k]; b[k] = b[r]; b[r] = tmp; }
  }
  for (int i = 0; i < N; ++i) {
    double acc = b[i];
    for (int k = 0; k < i; ++k) acc = acc - a[i * N + k] * b[k];
    b[i] = acc;
  }
  for (int i = N - 1; i >= 0; --i) {
    double acc = b[i];
    for (int k = N - 1; k > i; --k) acc = acc - a[i * N + k] * b[k];
    b[i] = acc / a[i * N + i];
  }
}

/* One trajectory of the rate equations by the Rosenbrock 4(3) method. */
static void ros4_traj(const dnet *g, const double *c, int64_t cld, double *y, const double *times,
                      int32_t n_times, double *out, int64_t out_ld, int64_t t, uint64_t *st,
                      const orc_ode_params *par, double *w, int *perm) {
  const int N = g->N;
  double *f0 = w, *fs = w + N, *ys = w + 2 * N, *u1 = w + 3 * N, *u2 = w + 4 * N,
         *u3 = w + 5 * N, *u4 = w + 6 * N, *yn = w + 7 * N, *a = w + 8 * N;
  double tt = 0.0;
  int s = 0;
  uint64_t acc = 0, rej = 0, status = 0;
  while (s < n_times && times[s] <= tt) {
    for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
    s++;
  }
  rhs(g, c, cld, y, f0);
  double d0 = 0.0, d1 = 0.0;
  for (int i = 0; i < N; ++i) {
    double sc = par->atol + par->rtol * fabs(y[i]);
    d0 = d0 + (y[i] / sc) * (y[i] / sc);
    d1 = d1 + (f0[i] / sc) * (f0[i] / sc);
  }
  d0 = sqrt(d0 / N);
  d1 = sqrt(d1 / N);
  double h = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  int last_rejected = 0;
  while (s < n_times) {
    if (acc + rej >= par->max_steps) { status |= ORC_ST_MAXSTEPS; break; }
    const double delta = times[s] - tt;
    const int clip = !(h < delta);
    const double hu = clip ? delta : h;
    const double ih = 1.0 / hu;
    const double gd = 1.0 / (RG * hu);
    /* W = (1/(gamma h)) I - J, factored */
    jacobian(g, c, cld, y, a);
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < N; ++k) a[i * N + k] = (i == k ? gd : 0.0) - a[i * N + k];
    lu_factor(N, a, perm);
    for (int i = 0; i < N; ++i) u1[i] = f0[i];
    lu_solve(N, a, perm, u1);
    for (int i = 0; i < N; ++i) ys[i] = y[i] + RA21 * u1[i];
    rhs(g, c, cld, ys, fs);
    for (int i = 0; i < N; ++i) u2[i] = fs[i] + (RC21 * u1[i]) * ih;
    lu_solve(N, a, perm, u2);
    for (int i = 0; i < N; ++i) ys[i] = y[i] + (RA31 * u1[i] + RA32 * u2[i]);
    rhs(g, c, cld, ys, fs);
    for (int i = 0; i < N; ++i) u3[i] = fs[i] + (RC31 * u1[i] + RC32 * u2[i]) * ih;
    lu_solve(N, a, perm, u3);
    for (int i = 0; i < N; ++i) u4[i] = fs[i] + (RC41 * u1[i] + RC42 * u2[i] + RC43 * u3[i]) * ih;
    lu_solve(N, a, perm, u4);
    double e2 = 0.0;
    for (int i = 0; i < N; ++i) {
      yn[i] = y[i] + (RM1 * u1[i] + RM2 * u2[i] + RM3 * u3[i] + RM4 * u4[i]);
      const double e = RE1 * u1[i] + RE2 * u2[i] + RE3 * u3[i] + RE4 * u4[i];
      const double ay = fabs(y[i]), an = fabs(yn[i]);
      const double sc = par->atol + par->rtol * (ay > an ? ay : an);
      e2 = e2 + (e / sc) * (e / sc);
    }
    const double en = sqrt(e2 / N);
    if (en <= 1.0) {
      double fac = en == 0.0 ? 5.0 : 0.9 * pow(en, -0.25);
      if (fac > 5.0) fac = 5.0;
      if (fac < 0.2) fac = 0.2;
      if (last_rejected && fac > 1.0) fac = 1.0;
      memcpy(y, yn, sizeof(double) * N);
      rhs(g, c, cld, y, f0);
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
      /* a NaN norm (a singular W, an overflow) is a rejection at the smallest factor */
      double fac = 0.9 * pow(en, -0.25);
      if (!(fac >= 0.2)) fac = 0.2;
      h = hu * fac;
      rej++;
      last_rejected = 1;
    }
  }
  while (s < n_times) {
    for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
    s++;
  }
  st[0] = acc;
  st[1] = rej;
  st[2] = 0;
  st[3] = status;
}

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
  if (par->method != ORC_ODE_DOPRI5 && par->method != ORC_ODE_ROS4) return ORC_E_ARG;
  dnet g;
  int err = dnet_build(net, &g);
  if (err) return err;
  const int N = g.N;
  if (par->method == ORC_ODE_ROS4) {
    double *rw = malloc(sizeof(double) * ((size_t)N * 9 + (size_t)N * N + (size_t)N));
    int *perm = malloc(sizeof(int) * (size_t)N);
    if (!rw || !perm) { free(rw); free(perm); dnet_free(&g); return ORC_E_NOMEM; }
    double *yv = rw + (size_t)N * 9 + (size_t)N * N;
    for (int64_t t = 0; t < n_traj; ++t) {
      for (int i = 0; i < N; ++i) yv[i] = (double)(x0_ld ? x0[(int64_t)i * x0_ld + t] : x0[i]);
      ros4_traj(&g, rates + t, rates_ld, yv, times, n_times, out, out_ld, t, stats + t * 4, par,
                rw, perm);
    }
    free(rw);
    free(perm);
    dnet_free(&g);
    return ORC_OK;
  }
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

/* a_j of discrete reaction j at y (stochastic mass-action form, floored at 0). */
static double hybrid_intensity(const dnet *g, int j, const double *c, int64_t cld,
                               const double *y) {
  double h;
  switch (g->kind[j]) {
    case 0: h = 1.0; break;
    case 1: h = y[g->ra[j]]; break;
    case 2: h = y[g->ra[j]] * y[g->rb[j]]; break;
    default: h = 0.5 * (y[g->ra[j]] * (y[g->ra[j]] - 1.0)); break;
  }
  double a = c[(int64_t)j * cld] * h;
  return a > 0.0 ? a : 0.0;
}

/* Flow f_y (continuous reactions, species-major in increasing j) and the
 * discrete intensity a0_D (increasing j) at y. */
static double hybrid_rhs(const dnet *g, const int32_t *cont, const double *c, int64_t cld,
                         const double *y, double *f) {
  for (int i = 0; i < g->N; ++i) f[i] = 0.0;
  double a0 = 0.0;
  for (int j = 0; j < g->M; ++j) {
    double h;
    if (cont[j]) {
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
    } else {
      a0 = a0 + hybrid_intensity(g, j, c, cld, y);
    }
  }
  return a0;
}

#define HYB_STREAM 0x80000000u
#define HYB_LOCATE_MAX 30
#define HYB_LOCATE_TOL 1e-12

/* One Dormand-Prince step of length hu from (y, L) with k1 = f(y), kl1 = a0_D(y):
 * yn, Ln, the stage derivatives k2..k7 (k7 = f(yn), kl[6] = a0_D(yn)) and the
 * error norm. */
static double hybrid_step(const dnet *g, const int32_t *cont, const double *c, int64_t cld,
                          const orc_hybrid_params *par, double hu, const double *y, double L,
                          const double *k1, double *k2, double *k3, double *k4, double *k5,
                          double *k6, double *k7, double *ys, double *yn, double *kl,
                          double *Ln) {
  const int N = g->N;
  for (int i = 0; i < N; ++i) ys[i] = y[i] + hu * (A21 * k1[i]);
  kl[1] = hybrid_rhs(g, cont, c, cld, ys, k2);
  for (int i = 0; i < N; ++i) ys[i] = y[i] + hu * (A31 * k1[i] + A32 * k2[i]);
  kl[2] = hybrid_rhs(g, cont, c, cld, ys, k3);
  for (int i = 0; i < N; ++i) ys[i] = y[i] + hu * (A41 * k1[i] + A42 * k2[i] + A43 * k3[i]);
  kl[3] = hybrid_rhs(g, cont, c, cld, ys, k4);
  for (int i = 0; i < N; ++i)
    ys[i] = y[i] + hu * (A51 * k1[i] + A52 * k2[i] + A53 * k3[i] + A54 * k4[i]);
  kl[4] = hybrid_rhs(g, cont, c, cld, ys, k5);
  for (int i = 0; i < N; ++i)
    ys[i] = y[i] + hu * (A61 * k1[i] + A62 * k2[i] + A63 * k3[i] + A64 * k4[i] + A65 * k5[i]);
  kl[5] = hybrid_rhs(g, cont, c, cld, ys, k6);
  for (int i = 0; i < N; ++i)
    yn[i] = y[i] + hu * (B1 * k1[i] + B3 * k3[i] + B4 * k4[i] + B5 * k5[i] + B6 * k6[i]);
  kl[6] = hybrid_rhs(g, cont, c, cld, yn, k7);
  *Ln = L + hu * (B1 * kl[0] + B3 * kl[2] + B4 * kl[3] + B5 * kl[4] + B6 * kl[5]);
  double e2 = 0.0;
  for (int i = 0; i < N; ++i) {
    double e = hu * (E1 * k1[i] + E3 * k3[i] + E4 * k4[i] + E5 * k5[i] + E6 * k6[i] + E7 * k7[i]);
    double ay = fabs(y[i]), an = fabs(yn[i]);
    double sc = par->atol + par->rtol * (ay > an ? ay : an);
    e2 = e2 + (e / sc) * (e / sc);
  }
  double en = sqrt(e2 / N);
  double el = hu * (E1 * kl[0] + E3 * kl[2] + E4 * kl[3] + E5 * kl[4] + E6 * kl[5] + E7 * kl[6]);
  double al = fabs(L), anl = fabs(*Ln);
  double ll = fabs(el) / (par->atol + par->rtol * (al > anl ? al : anl));
  return ll > en ? ll : en;
}

int orc_hybrid_run(const orc_net_desc *net, const int32_t *cont, const double *rates,
                   int64_t rates_ld, const int32_t *x0, int64_t x0_ld, const double *times,
                   int32_t n_times, int64_t traj0, int64_t n_traj, double *out, int64_t out_ld,
                   uint64_t *stats, const orc_hybrid_params *par) {
  if (!net || !cont || !rates || !x0 || !times || !out || !stats || !par) return ORC_E_ARG;
  if (n_times <= 0 || n_traj < 0 || traj0 < 0 || !(par->rtol > 0.0) || !(par->atol > 0.0) ||
      par->max_steps < 1)
    return ORC_E_ARG;
  for (int s = 0; s < n_times; ++s) {
    if (!(times[s] >= 0.0) || !isfinite(times[s])) return ORC_E_ARG;
    if (s > 0 && !(times[s] > times[s - 1])) return ORC_E_ARG;
  }
  dnet g;
  int err = dnet_build(net, &g);
  if (err) return err;
  const int N = g.N;
  double *w = malloc(sizeof(double) * (size_t)N * 12);
  if (!w) { dnet_free(&g); return ORC_E_NOMEM; }
  double *y = w, *yn = w + N, *k1 = w + 2 * N, *k2 = w + 3 * N, *k3 = w + 4 * N, *k4 = w + 5 * N,
         *k5 = w + 6 * N, *k6 = w + 7 * N, *k7 = w + 8 * N, *ys = w + 9 * N, *ye = w + 10 * N,
         *ke = w + 11 * N;
  const uint32_t key[2] = {(uint32_t)par->seed, (uint32_t)(par->seed >> 32)};
  for (int64_t t = 0; t < n_traj; ++t) {
    const double *c = rates + t;
    const uint32_t tr = (uint32_t)(traj0 + t);
    for (int i = 0; i < N; ++i) y[i] = (double)(x0_ld ? x0[(int64_t)i * x0_ld + t] : x0[i]);
    double tt = 0.0, L = 0.0, xi, u;
    uint32_t njump = 0;
    {
      uint32_t ctr[4] = {tr, 0u, 0u, HYB_STREAM}, o[4];
      orc_philox4x32_10(ctr, key, o);
      xi = -log(1.0 - orc_u53(o[0], o[1]));
      u = orc_u53(o[2], o[3]);
    }
    int s = 0;
    uint64_t acc = 0, rej = 0, status = 0;
    while (s < n_times && times[s] <= tt) {
      for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
      s++;
    }
    double kl[7];
    kl[0] = hybrid_rhs(&g, cont, c, rates_ld, y, k1);
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
      double Ln;
      double en = hybrid_step(&g, cont, c, rates_ld, par, hu, y, L, k1, k2, k3, k4, k5, k6, k7,
                              ys, yn, kl, &Ln);
      if (!(en <= 1.0)) {
        double fac = 0.9 * pow(en, -0.2);
        if (fac < 0.2) fac = 0.2;
        h = hu * fac;
        rej++;
        last_rejected = 1;
        continue;
      }
      double fac = en == 0.0 ? 5.0 : 0.9 * pow(en, -0.2);
      if (fac > 5.0) fac = 5.0;
      if (fac < 0.2) fac = 0.2;
      if (last_rejected && fac > 1.0) fac = 1.0;
      last_rejected = 0;
      acc++;
      if (Ln < xi) {  /* no jump inside the step */
        memcpy(y, yn, sizeof(double) * N);
        memcpy(k1, k7, sizeof(double) * N);
        kl[0] = kl[6];
        L = Ln;
        if (clip) tt = times[s];
        else tt = tt + hu;
        h = hu * fac;
        while (s < n_times && times[s] <= tt) {
          for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
          s++;
        }
        continue;
      }
      /* The jump lies in (0, hu]: the Illinois variant of regula falsi on the
       * step length over the bracket [0, hu] of g = L - xi, each trial a full
       * step from the same start, until |g| <= tol * (1 + xi). */
      double he = 0.0;
      memcpy(ye, y, sizeof(double) * N);
      if (xi - L > 0.0) {
        double hl = 0.0, gl = L - xi, hr = hu, gr = Ln - xi;
        int side = 0;
        for (int r = 0; r < HYB_LOCATE_MAX; ++r) {
          he = hl - gl * ((hr - hl) / (gr - gl));
          double kle[7], Le;
          kle[0] = kl[0];
          (void)hybrid_step(&g, cont, c, rates_ld, par, he, y, L, k1, k2, k3, k4, k5, k6, ke, ys,
                            ye, kle, &Le);
          rej++;
          double ge = Le - xi;
          if (fabs(ge) <= HYB_LOCATE_TOL * (1.0 + xi)) break;
          if (ge < 0.0) {
            hl = he; gl = ge;
            if (side < 0) gr = 0.5 * gr;
            side = -1;
          } else {
            hr = he; gr = ge;
            if (side > 0) gl = 0.5 * gl;
            side = 1;
          }
        }
      }
      memcpy(y, ye, sizeof(double) * N);
      tt = tt + he;
      h = hu * fac;
      while (s < n_times && times[s] <= tt) {  /* samples take the pre-jump state */
        for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
        s++;
      }
      /* fire the discrete reaction chosen at the jump state */
      double a0 = 0.0;
      for (int j = 0; j < g.M; ++j)
        if (!cont[j]) a0 = a0 + hybrid_intensity(&g, j, c, rates_ld, y);
      if (a0 > 0.0) {
        double r = u * a0, acc_a = 0.0;
        int pick = -1, last = -1;
        for (int j = 0; j < g.M && pick < 0; ++j) {
          if (cont[j]) continue;
          double a = hybrid_intensity(&g, j, c, rates_ld, y);
          acc_a = acc_a + a;
          if (a > 0.0) last = j;
          if (r < acc_a) pick = j;
        }
        if (pick < 0) pick = last;
        for (int i = 0; i < N; ++i) y[i] = y[i] + (double)g.nu[(size_t)pick * N + i];
      }
      njump++;
      {
        uint32_t ctr[4] = {tr, njump, 0u, HYB_STREAM}, o[4];
        orc_philox4x32_10(ctr, key, o);
        xi = -log(1.0 - orc_u53(o[0], o[1]));
        u = orc_u53(o[2], o[3]);
      }
      L = 0.0;
      kl[0] = hybrid_rhs(&g, cont, c, rates_ld, y, k1);
    }
    while (s < n_times) {
      for (int i = 0; i < N; ++i) out[((int64_t)s * N + i) * out_ld + t] = y[i];
      s++;
    }
    stats[t * 4 + 0] = acc;
    stats[t * 4 + 1] = rej;
    stats[t * 4 + 2] = njump;
    stats[t * 4 + 3] = status;
  }
  free(w);
  dnet_free(&g);
  return ORC_OK;
}
