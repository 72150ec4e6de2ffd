"""Pins of the deterministic (reaction-rate equation) oracle: closed forms,
an independent integrator, and convergence with the tolerance."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_1309_7695_amd import gen


def _ode(net, rates, x0, times, runs=3, **kw):
    r = np.repeat(np.asarray(rates, float)[:, None], runs, axis=1)
    out, st = oracle.ode_run(net, r, np.asarray(x0, np.int32), np.asarray(times, float), **kw)
    return out, st


def test_decay_exponential():
    times = gen.sample_times(5.0, 11)
    out, st = _ode(gen.decay_network(), [0.7], [1000], times, rtol=1e-10, atol=1e-10)
    want = 1000 * np.exp(-0.7 * times)
    assert np.allclose(out[:, 0, 0], want, rtol=1e-8, atol=0)
    assert np.all(st[:, 3] == 0) and np.all(st[:, 0] > 0)


def test_source_is_linear_exactly():
    times = gen.sample_times(3.0, 7)
    out, _ = _ode(gen.source_network(), [2.5], [4], times, rtol=1e-6, atol=1e-6)
    assert np.allclose(out[:, 0, 0], 4 + 2.5 * times, rtol=1e-13, atol=1e-12)


def test_birth_death_relaxation():
    times = gen.sample_times(4.0, 9)
    k1, k2, y0 = 30.0, 1.5, 2.0
    out, _ = _ode(gen.birth_death_network(), [k1, k2], [int(y0)], times, rtol=1e-10, atol=1e-10)
    want = k1 / k2 + (y0 - k1 / k2) * np.exp(-k2 * times)
    assert np.allclose(out[:, 0, 0], want, rtol=1e-8)


def test_dimerization_pins_half_square():
    # 2A -> B with rate c*y^2/2: dy/dt = -c y^2, y = y0 / (1 + c y0 t)
    times = gen.sample_times(2.0, 5)
    c, y0 = 0.01, 300.0
    out, _ = _ode(gen.dimerization_network(), [c], [int(y0), 0], times, rtol=1e-10, atol=1e-10)
    want = y0 / (1 + c * y0 * times)
    assert np.allclose(out[:, 0, 0], want, rtol=1e-8)
    assert np.allclose(out[:, 0, 0] + 2 * out[:, 1, 0], y0, rtol=1e-12)


def test_isomerization_closed_form():
    times = gen.sample_times(3.0, 7)
    k1, k2, n = 1.3, 0.4, 50.0
    out, _ = _ode(gen.isomerization_network(), [k1, k2], [int(n), 0], times, rtol=1e-10,
                  atol=1e-10)
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


def test_random_network_against_independent_integrator_and_convergence():
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
        out, _ = _ode(net, rates, x0, times, runs=1, rtol=tol, atol=tol)
        errs.append(np.max(np.abs(out[:, :, 0] - sol.y.T) / (1 + np.abs(sol.y.T))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-7


def test_maxsteps_and_rejections():
    out, st = _ode(gen.decay_network(), [50.0], [1000], [0.0, 10.0], rtol=1e-12, atol=1e-12,
                   max_steps=5)
    assert np.all(st[:, 3] == oracle.ST_MAXSTEPS)
    assert np.all(st[:, 0] + st[:, 1] == 5)
