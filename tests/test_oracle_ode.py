"""Pins of the deterministic (reaction-rate equation) oracle: closed forms,
an independent integrator, and convergence with the tolerance, for both the
Dormand-Prince 5(4) pair and the Rosenbrock 4(3) method; for the latter also
its tableau's order conditions, its stability function on a linear step, the
order of its local error and a stiff network against scipy's Radau."""
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_1309_7695_amd import gen


def _ode(net, rates, x0, times, runs=3, **kw):
    r = np.repeat(np.asarray(rates, float)[:, None], runs, axis=1)
    out, st = oracle.ode_run(net, r, np.asarray(x0, np.int32), np.asarray(times, float), **kw)
    return out, st


@pytest.mark.parametrize("method", ["dopri5", "ros4"])
def test_decay_exponential(method):
    times = gen.sample_times(5.0, 11)
    out, st = _ode(gen.decay_network(), [0.7], [1000], times, rtol=1e-10, atol=1e-10,
                   method=method)
    want = 1000 * np.exp(-0.7 * times)
    assert np.allclose(out[:, 0, 0], want, rtol=1e-8, atol=0)
    assert np.all(st[:, 3] == 0) and np.all(st[:, 0] > 0)


@pytest.mark.parametrize("method", ["dopri5", "ros4"])
def test_source_is_linear_exactly(method):
    times = gen.sample_times(3.0, 7)
    out, _ = _ode(gen.source_network(), [2.5], [4], times, rtol=1e-6, atol=1e-6, method=method)
    assert np.allclose(out[:, 0, 0], 4 + 2.5 * times, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("method", ["dopri5", "ros4"])
def test_birth_death_relaxation(method):
    times = gen.sample_times(4.0, 9)
    k1, k2, y0 = 30.0, 1.5, 2.0
    out, _ = _ode(gen.birth_death_network(), [k1, k2], [int(y0)], times, rtol=1e-10, atol=1e-10,
                  method=method)
    want = k1 / k2 + (y0 - k1 / k2) * np.exp(-k2 * times)
    assert np.allclose(out[:, 0, 0], want, rtol=1e-8)


@pytest.mark.parametrize("method", ["dopri5", "ros4"])
def test_dimerization_pins_half_square(method):
    # 2A -> B with rate c*y^2/2: dy/dt = -c y^2, y = y0 / (1 + c y0 t)
    times = gen.sample_times(2.0, 5)
    c, y0 = 0.01, 300.0
    out, _ = _ode(gen.dimerization_network(), [c], [int(y0), 0], times, rtol=1e-10, atol=1e-10,
                  method=method)
    want = y0 / (1 + c * y0 * times)
    assert np.allclose(out[:, 0, 0], want, rtol=1e-8)
    assert np.allclose(out[:, 0, 0] + 2 * out[:, 1, 0], y0, rtol=1e-12)


@pytest.mark.parametrize("method", ["dopri5", "ros4"])
def test_isomerization_closed_form(method):
    times = gen.sample_times(3.0, 7)
    k1, k2, n = 1.3, 0.4, 50.0
    out, _ = _ode(gen.isomerization_network(), [k1, k2], [int(n), 0], times, rtol=1e-10,
                  atol=1e-10, method=method)
    eq = n * k2 / (k1 + k2)
    want = eq + (n - eq) * np.exp(-(k1 + k2) * times)
    assert np.allclose(out[:, 0, 0], want, rtol=1e-8)


def test_enzyme_against_independent_integrator():
    w = gen.enzyme_workload(n_traj=4)
    out, st = oracle.ode_run(w.net, w.rates, w.x0, w.times, rtol=1e-9, atol=1e-9)
    for t in range(4):
        k1, km1, k2 = w.rates[:, t]

        def f(_, y):
            e, s, es, p = y
            r0, r1, r2 = k1 * e * s, km1 * es, k2 * es
            return [-r0 + r1 + r2, -r0 + r1, r0 - r1 - r2, r2]

        sol = solve_ivp(f, (0, w.times[-1]), w.x0.astype(float), method="DOP853", rtol=1e-12,
                        atol=1e-12, t_eval=w.times)
        assert np.allclose(out[:, :, t], sol.y.T, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("method", ["dopri5", "ros4"])
def test_random_network_against_independent_integrator_and_convergence(method):
    net = gen.random_network(11, 8, 14)
    rng = np.random.default_rng(2)
    rates = gen.log_uniform(rng, 1e-3, 0.5, 14)
    x0 = rng.integers(10, 200, size=8).astype(np.int32)
    times = gen.sample_times(5.0, 6)
    R = np.zeros((8, 14), dtype=np.int64)
    P = np.zeros((8, 14), dtype=np.int64)
    for j in range(14):
        for s, c in net.reactants[j]:
            R[s, j] = c
        for s, c in net.products[j]:
            P[s, j] = c
    nu = P - R

    def f(_, y):
        a = np.empty(14)
        for j in range(14):
            h = 1.0
            for s, c in net.reactants[j]:
                h *= y[s] ** c / (2.0 if c == 2 else 1.0)
            a[j] = rates[j] * h
        return nu @ a

    sol = solve_ivp(f, (0, 5.0), x0.astype(float), method="DOP853", rtol=1e-12, atol=1e-12,
                    t_eval=times)
    errs = []
    for tol in (1e-4, 1e-7, 1e-10):
        out, _ = _ode(net, rates, x0, times, runs=1, rtol=tol, atol=tol, method=method)
        errs.append(np.max(np.abs(out[:, :, 0] - sol.y.T) / (1 + np.abs(sol.y.T))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-7


@pytest.mark.parametrize("method", ["dopri5", "ros4"])
def test_maxsteps_and_rejections(method):
    out, st = _ode(gen.decay_network(), [50.0], [1000], [0.0, 10.0], rtol=1e-12, atol=1e-12,
                   max_steps=5, method=method)
    assert np.all(st[:, 3] == oracle.ST_MAXSTEPS)
    assert np.all(st[:, 0] + st[:, 1] == 5)


# ---- the Rosenbrock 4(3) method ------------------------------------------------
# Shampine's gamma = 1/2 parameter set (ACM Trans. Math. Softw. 8 (1982) 93) in
# the transformed form (Hairer and Wanner, Solving ODEs II, Sec. IV.7): stage
# arguments a_ij, stage corrections c_ij / h, solution weights m_i.  The fourth
# stage reuses the third stage's argument.
ROS_GAMMA = Fraction(1, 2)
ROS_A = {(1, 0): Fraction(2), (2, 0): Fraction(48, 25), (2, 1): Fraction(6, 25),
         (3, 0): Fraction(48, 25), (3, 1): Fraction(6, 25)}
ROS_C = {(1, 0): Fraction(-8), (2, 0): Fraction(372, 25), (2, 1): Fraction(12, 5),
         (3, 0): Fraction(-112, 125), (3, 1): Fraction(-54, 125), (3, 2): Fraction(-2, 5)}
ROS_M = [Fraction(19, 9), Fraction(1, 2), Fraction(25, 108), Fraction(125, 108)]
ROS_E = [Fraction(17, 54), Fraction(7, 36), Fraction(0), Fraction(125, 108)]


def _ros_standard_form():
    """(alpha, Gamma, b, b_hat) of the standard form k_i = h f(y + sum alpha_ij k_j)
    + h J sum gamma_ij k_j, y1 = y + sum b_i k_i, from the transformed
    coefficients: Gamma^-1 = diag(1/gamma) - C, alpha = A Gamma, b = m Gamma,
    and the embedded weights from m - e."""
    n = 4
    gi = [[(1 / ROS_GAMMA if i == j else Fraction(0)) - ROS_C.get((i, j), Fraction(0))
           for j in range(n)] for i in range(n)]
    G = [[Fraction(0)] * n for _ in range(n)]
    for j in range(n):  # lower-triangular inverse by forward substitution
        for i in range(j, n):
            acc = Fraction(1) if i == j else Fraction(0)
            for k in range(j, i):
                acc -= gi[i][k] * G[k][j]
            G[i][j] = acc / gi[i][i]
    A = [[ROS_A.get((i, j), Fraction(0)) for j in range(n)] for i in range(n)]
    alpha = [[sum(A[i][k] * G[k][j] for k in range(n)) for j in range(n)] for i in range(n)]
    b = [sum(ROS_M[k] * G[k][j] for k in range(n)) for j in range(n)]
    bh = [sum((ROS_M[k] - ROS_E[k]) * G[k][j] for k in range(n)) for j in range(n)]
    return alpha, G, b, bh


def _order_defects(alpha, G, b):
    """Residuals of the eight Rosenbrock order conditions up to order 4
    (Hairer and Wanner, Solving ODEs II, Table IV.7.1), with
    beta_ij = alpha_ij + gamma_ij below the diagonal."""
    n, g = 4, ROS_GAMMA
    beta = [[alpha[i][j] + (G[i][j] if j < i else 0) for j in range(n)] for i in range(n)]
    al = [sum(alpha[i]) for i in range(n)]
    bp = [sum(beta[i]) for i in range(n)]
    R = range(n)
    return [
        sum(b) - 1,
        sum(b[i] * bp[i] for i in R) - (Fraction(1, 2) - g),
        sum(b[i] * al[i] ** 2 for i in R) - Fraction(1, 3),
        sum(b[i] * beta[i][j] * bp[j] for i in R for j in R) - (Fraction(1, 6) - g + g * g),
        sum(b[i] * al[i] ** 3 for i in R) - Fraction(1, 4),
        sum(b[i] * al[i] * alpha[i][j] * bp[j] for i in R for j in R) - (Fraction(1, 8) - g / 3),
        sum(b[i] * beta[i][j] * al[j] ** 2 for i in R for j in R) - (Fraction(1, 12) - g / 3),
        sum(b[i] * beta[i][j] * beta[j][k] * bp[k] for i in R for j in R for k in R)
        - (Fraction(1, 24) - g / 2 + Fraction(3, 2) * g * g - g ** 3),
    ]


def test_ros4_tableau_has_orders_four_and_three():
    alpha, G, b, bh = _ros_standard_form()
    assert all(d == 0 for d in _order_defects(alpha, G, b))
    emb = _order_defects(alpha, G, bh)
    assert all(d == 0 for d in emb[:4]) and any(d != 0 for d in emb[4:])


def _stability(z):
    """R(z) = 1 + z b^T (I - z B)^-1 1 with B = alpha + Gamma: one step of the
    method on y' = lambda y multiplies y by R(h lambda)."""
    alpha, G, b, _ = _ros_standard_form()
    B = np.array([[float(alpha[i][j] + G[i][j]) for j in range(4)] for i in range(4)])
    return 1.0 + z * np.array([float(v) for v in b]) @ np.linalg.solve(np.eye(4) - z * B,
                                                                     np.ones(4))


@pytest.mark.parametrize("a0,b0,T", [(500, 501, 0.5), (5000, 5001, 50.0)])
def test_ros4_linear_step_is_the_stability_function(a0, b0, T):
    # A <-> B with unit rates: the deviation from the equilibrium (a0+b0)/2 is the
    # eigenvector of eigenvalue -2, so one step of length T scales it by R(-2T);
    # starting near equilibrium makes the first step longer than T, so the step
    # is clipped to the sample time (z = -1, and z = -100 in the stiff range).
    out, st = oracle.ode_run(gen.isomerization_network(), np.array([[1.0], [1.0]]),
                             np.array([a0, b0], np.int32), np.array([0.0, T]), rtol=1e-2,
                             atol=1e-2, max_steps=1, method="ros4")
    assert st[0, 0] == 1 and st[0, 3] == 0
    eq = (a0 + b0) / 2
    want = eq + _stability(-2.0 * T) * (a0 - eq)
    assert abs(out[1, 0, 0] - want) <= 1e-12 * eq
    assert abs(out[1, 1, 0] - (a0 + b0 - want)) <= 1e-12 * eq
    # the method is A-stable but not L-stable: R(-inf) = 1/3
    assert abs(_stability(-1e12) - 1.0 / 3.0) < 1e-9


def test_ros4_local_error_is_fifth_order():
    # 2A -> B: y' = -c y^2, y(T) = y0 / (1 + c y0 T).  One step of an order-4
    # method errs by O(T^5): halving T divides the error by about 32 (an
    # order-3 method would give about 16).
    c, y0 = 0.01, 300
    errs = []
    for T in (1 / 300, 1 / 600):
        out, st = oracle.ode_run(gen.dimerization_network(), np.array([[c]]),
                                 np.array([y0, 10000], np.int32), np.array([0.0, T]),
                                 rtol=1e-2, atol=1e-2, max_steps=1, method="ros4")
        assert st[0, 0] == 1 and st[0, 3] == 0
        errs.append(out[1, 0, 0] - y0 / (1 + c * y0 * T))
    assert 24.0 < errs[0] / errs[1] < 40.0


def _mass_action_rhs(net, rates):
    N, M = net.n_species, len(net.reactants)
    R = np.zeros((N, M))
    P = np.zeros((N, M))
    for j in range(M):
        for s_, c_ in net.reactants[j]:
            R[s_, j] = c_
        for s_, c_ in net.products[j]:
            P[s_, j] = c_
    nu = P - R

    def f(_, y):
        a = np.empty(M)
        for j in range(M):
            h = 1.0
            for s_, c_ in net.reactants[j]:
                h *= y[s_] ** c_ / (2.0 if c_ == 2 else 1.0)
            a[j] = rates[j] * h
        return nu @ a

    def jac(_, y):
        D = np.zeros((M, N))
        for j in range(M):
            r = net.reactants[j]
            if len(r) == 1:
                s_, c_ = r[0]
                D[j, s_] = rates[j] * (y[s_] if c_ == 2 else 1.0)
            elif len(r) == 2:
                (a_, _), (b_, _) = r
                D[j, a_] = rates[j] * y[b_]
                D[j, b_] = rates[j] * y[a_]
        return nu @ D

    return f, jac


def test_ros4_stiff_network_against_radau():
    # the stiff 30x80 network (rates over eight decades): scipy's Radau IIA with
    # its own Jacobian at rtol 1e-11 is the reference
    w = gen.stiff_workload(n_traj=3)
    out, st = oracle.ode_run(w.net, w.rates, w.x0, w.times, rtol=1e-6, atol=1e-6, method="ros4")
    assert np.all(st[:, 3] == 0)
    for t in range(3):
        f, jac = _mass_action_rhs(w.net, w.rates[:, t])
        sol = solve_ivp(f, (0, w.times[-1]), w.x0.astype(float), method="Radau", jac=jac,
                        rtol=1e-11, atol=1e-9, t_eval=w.times)
        assert sol.status == 0
        ref = sol.y.T
        assert np.max(np.abs(out[:, :, t] - ref) / (1 + np.abs(ref))) < 2e-5


def test_ros4_needs_far_fewer_steps_than_dopri5_on_the_stiff_network():
    w = gen.stiff_workload(n_traj=4)
    _, st_e = oracle.ode_run(w.net, w.rates, w.x0, w.times, rtol=1e-6, atol=1e-6)
    _, st_r = oracle.ode_run(w.net, w.rates, w.x0, w.times, rtol=1e-6, atol=1e-6, method="ros4")
    assert np.all(st_r[:, :2].sum(1) * 3 < st_e[:, :2].sum(1))


def test_ros4_keeps_linear_invariants():
    # every stage lies in the range of the stoichiometry, so E + ES and S + ES + P
    # stay at their initial values up to rounding
    w = gen.enzyme_workload(n_traj=8)
    out, _ = oracle.ode_run(w.net, w.rates, w.x0, w.times, rtol=1e-6, atol=1e-6, method="ros4")
    e_tot = out[:, 0, :] + out[:, 2, :]
    s_tot = out[:, 1, :] + out[:, 2, :] + out[:, 3, :]
    assert np.allclose(e_tot, w.x0[0] + w.x0[2], rtol=1e-12, atol=0)
    assert np.allclose(s_tot, w.x0[1] + w.x0[2] + w.x0[3], rtol=1e-12, atol=0)
