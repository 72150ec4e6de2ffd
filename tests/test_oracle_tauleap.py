"""Pins of the oracle's tau-leaping path: exact special cases, a deterministic
leap sequence, the all-critical reduction to SSA, invariants, determinism and
the status rules."""
import numpy as np
import pytest
from scipy import stats as sst
from scipy.integrate import solve_ivp

import oracle
from paper_1309_7695_amd import gen
from tests.stats_util import chi2_pvalue, z_mean, z_var


def _run(net, rates_nominal, x0, times, seed, runs, **kw):
    rates = np.repeat(np.asarray(rates_nominal, dtype=float)[:, None], runs, axis=1)
    kw.setdefault("threads", 8)
    return oracle.run(net, rates, np.asarray(x0, dtype=np.int32), np.asarray(times, float),
                      seed=seed, **kw)


@pytest.mark.parametrize("c", [3.0, 40.0])
def test_source_is_exactly_poisson(c):
    # 0 -> A has no reactant species, so tau' is infinite and every leap runs to
    # the next sample time: X(t) ~ Poisson(c t) exactly (both Poisson branches)
    net = gen.source_network()
    times = [0.0, 0.5, 1.0, 2.0]
    out, st, _ = _run(net, [c], [0], times, seed=21, runs=100000)
    assert np.all(st[:, 0] == 3) and np.all(st[:, 1] == 0) and np.all(st[:, 2] == 0)
    for s, t in enumerate(times[1:], start=1):
        lam = c * t
        pmf = sst.poisson.pmf(np.arange(int(lam + 12 * np.sqrt(lam) + 30)), lam)
        assert chi2_pvalue(out[s, 0], pmf) > 1e-3
        assert z_mean(out[s, 0], lam) < 4


def test_catalytic_production_is_exactly_poisson():
    # A -> A + B never changes A, so mu_A = 0 and tau' is infinite:
    # B(t) ~ Poisson(c A0 t)
    net = gen.catalytic_network()
    c, A0 = 0.7, 20
    times = [0.0, 0.25, 1.0]
    out, st, _ = _run(net, [c], [A0, 0], times, seed=22, runs=100000)
    assert np.all(out[:, 0] == A0)
    for s, t in enumerate(times[1:], start=1):
        lam = c * A0 * t
        pmf = sst.poisson.pmf(np.arange(int(lam + 12 * np.sqrt(lam) + 30)), lam)
        assert chi2_pvalue(out[s, 1], pmf) > 1e-3


def test_decay_deterministic_leap_sequence():
    # x0 = 1e5, k = 1, eps = 0.03: b = eps x, mu = -x, sigma^2 = x, so
    # tau' = min(eps, eps^2 x) = 0.03 while x >= 34, and the SSA switch needs
    # x < 10/0.03.  Every 0.1 interval takes leaps 0.03, 0.03, 0.03 and a
    # clipped one of about 0.01: exactly 80 leaps to t = 2.
    net = gen.decay_network()
    times = gen.sample_times(2.0, 21)
    runs = 20000
    out, st, _ = _run(net, [1.0], [100000], times, seed=23, runs=runs)
    assert np.all(st[:, 0] == 80)
    assert np.all(st[:, 1] == 0) and np.all(st[:, 2] == 0)
    # moments by the leap recursion: m' = (1-tau) m, v' = (1-tau)^2 v + tau m
    m, v = 1e5, 0.0
    t = 0.0
    for s in range(1, 21):
        taus = [0.03, 0.03, 0.03, times[s] - (times[s - 1] + 0.09)]
        for tau in taus:
            v = (1 - tau) ** 2 * v + tau * m
            m = (1 - tau) * m
        assert z_mean(out[s, 0], m) < 4.5
        assert z_var(out[s, 0], v) < 4.5
    assert abs(m - 13152.5) < 1.0   # the tau-leap mean (CME mean is 13533.5)


@pytest.mark.parametrize("name,rates,x0", [
    ("enzyme", [0.3, 0.5, 0.7], [2, 5, 0, 0]),
    ("isomerization", [1.0, 0.5], [8, 0]),
])
def test_all_critical_reduction_is_bitwise_ssa(name, rates, x0):
    # with only {0, t_end} as sample times, every leap is one critical firing
    # drawn from the same counter slots as an SSA event
    net = getattr(gen, name + "_network")()
    times = [0.0, 5.0]
    runs = 20000
    out_l, st_l, _ = _run(net, rates, x0, times, seed=24, runs=runs, method="tauleap")
    out_s, st_s, _ = _run(net, rates, x0, times, seed=24, runs=runs, method="ssa")
    assert np.array_equal(out_l, out_s)
    alive = (st_s[:, 3] & oracle.ST_ABSORBED) == 0
    # the final leap to t_end is one extra (clipped, event-free) leap
    assert np.array_equal(st_l[alive, 0], st_s[alive, 1] + 1)
    assert np.array_equal(st_l[~alive, 0], st_s[~alive, 1])


def test_epsilon_convergence_to_ssa_moments():
    # birth-death k1 = 1000, k2 = 1: stationary Poisson(1000).  Tau-leap variance
    # inflation shrinks as eps -> 0 (the leap scheme's bias)
    net = gen.birth_death_network()
    times = [0.0, 10.0]
    ref, _, _ = _run(net, [1000.0, 1.0], [1000], times, seed=25, runs=4000, method="ssa")
    ratios = []
    for eps in (0.1, 0.03, 0.01):
        out, st, _ = _run(net, [1000.0, 1.0], [1000], times, seed=26, runs=4000, eps=eps)
        ratios.append(out[1, 0].var() / out[1, 0].mean())
    assert abs(ref[1, 0].var() / ref[1, 0].mean() - 1.0) < 0.1
    assert ratios[0] > ratios[2]
    assert abs(ratios[2] - 1.0) < 0.1


def test_kurtz_limit_enzyme():
    # Omega-scaled enzyme: x0 = Omega (1, 5, 0, 0), k1 -> k1/Omega; P/Omega
    # approaches the reaction-rate equation solution as Omega grows (paper,
    # Methods section: thermodynamic limit)
    k1, km1, k2 = 2.0, 0.5, 1.0
    tend = 2.0

    def rre(t, y):
        e, s, es, p = y
        r0, r1, r2 = k1 * e * s, km1 * es, k2 * es
        return [-r0 + r1 + r2, -r0 + r1, r0 - r1 - r2, r2]

    sol = solve_ivp(rre, (0, tend), [1.0, 5.0, 0.0, 0.0], rtol=1e-10, atol=1e-12)
    p_det = sol.y[3, -1]
    errs = []
    net = gen.enzyme_network()
    for om in (4, 40, 400):
        out, _, _ = _run(net, [k1 / om, km1, k2], [om, 5 * om, 0, 0], [0.0, tend], seed=27,
                         runs=3000)
        errs.append(abs(out[1, 3].mean() / om - p_det))
    assert errs[0] > errs[2]
    assert errs[2] < 0.02


def test_conservation_and_nonnegativity_enzyme_workload():
    w = gen.enzyme_workload(n_traj=256)
    out, st, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=1, threads=8)
    assert out.min() >= 0
    assert np.all(out[0] == w.x0[:, None])
    E, S, ES, P = out[:, 0], out[:, 1], out[:, 2], out[:, 3]
    assert np.all(E + ES == 100)
    assert np.all(S + ES + P == 500)


def test_random_network_mass_never_grows_without_sources():
    net, mass = gen.random_network(77, 12, 20, frac_first=0.5, frac_second=0.5,
                                   return_mass=True)
    rng = np.random.default_rng(1)
    runs = 64
    rates = gen.log_uniform(rng, 1e-3, 1.0, (20, runs))
    x0 = rng.integers(0, 200, size=12).astype(np.int32)
    out, st, _ = oracle.run(net, rates, x0, gen.sample_times(5.0, 21), seed=3)
    tot = np.einsum("i,sit->st", mass, out.astype(np.int64))
    assert np.all(np.diff(tot, axis=0) <= 0)
    assert out.min() >= 0


def test_subset_equals_slice_and_threads_invariant():
    w = gen.synthetic_workload(n_traj=64, n_species=10, n_reactions=20, t_end=5.0,
                               n_samples=11)
    full, sf, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=5)
    part, sp, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=5, traj_range=(17, 40))
    assert np.array_equal(full[:, :, 17:40], part)
    assert np.array_equal(sf[17:40], sp)
    thr, st_, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=5, threads=5)
    assert np.array_equal(full, thr) and np.array_equal(sf, st_)
    other, _, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=6)
    assert not np.array_equal(full, other)


def test_status_absorbed_fills_remaining_samples():
    net = gen.decay_network()
    out, st, _ = _run(net, [5.0], [3], gen.sample_times(10.0, 11), seed=30, runs=100)
    assert np.all(st[:, 3] == oracle.ST_ABSORBED)
    assert np.all(out[-1, 0] == 0)


def test_status_maxsteps_freezes_state():
    net = gen.birth_death_network()
    out, st, _ = _run(net, [10.0, 0.1], [0], gen.sample_times(100.0, 11), seed=31, runs=50,
                      max_steps=7, method="ssa")
    assert np.all(st[:, 3] == oracle.ST_MAXSTEPS)
    assert np.all(st[:, 1] == 7)
    last = out[:, 0, :]
    assert np.all(last[-1] == last[-2])


def test_status_overflow_on_runaway_source():
    net = gen.source_network()
    out, st, _ = _run(net, [1e12], [0], [0.0, 1.0], seed=32, runs=8)
    assert np.all(st[:, 3] == oracle.ST_OVERFLOW)
    assert np.all(out[1, 0] == 0)


def test_rejections_happen_and_stay_nonnegative():
    # a loose leap condition (eps = 0.9), no critical reactions (n_c = 0) and no
    # SSA switch make negative proposals common; they must be rejected
    net = gen.reversible_dimer_network()
    out, st, _ = _run(net, [0.5, 5.0], [60, 20], gen.sample_times(5.0, 11), seed=33,
                      runs=2000, eps=0.9, n_c=0, ssa_factor=0.0)
    assert out.min() >= 0
    assert np.all(out[:, 0] + 2 * out[:, 1] == 100)
    assert st[:, 2].sum() > 0


def test_invalid_arguments():
    net = gen.decay_network()
    with pytest.raises(RuntimeError):
        _run(net, [1.0], [1], [0.0, 0.0], seed=1, runs=2)     # not increasing
    with pytest.raises(RuntimeError):
        _run(net, [1.0], [1], [0.0, 1.0], seed=1, runs=2, ssa_burst=0)
    tri = gen.make_network(1, [([(0, 3)], [])])
    with pytest.raises(RuntimeError):
        _run(tri, [1.0], [5], [0.0, 1.0], seed=1, runs=2)     # order 3


@pytest.mark.parametrize("kind", ["first", "pair", "dimer"])
def test_single_leap_pins_g_factor(kind):
    # With max_steps = 1 the run stops after its first attempt, so the second
    # sample holds the state after exactly one leap of size tau'.  With eps = 0.5
    # the leap condition bound b = max(eps x / g, 1) exceeds 1 and the CGP g
    # factor (1 for first order, 2 for A + B, 2 + 1/(x-1) for 2A) sets tau':
    # tau' = min(b/|mu|, b^2/sigma^2).  A rejected attempt leaves x0.
    eps, x = 0.5, 6
    if kind == "first":
        net = gen.decay_network(); x0 = [x]; c = 1.0
        a, nu, g = c * x, -1, 1.0
    elif kind == "pair":
        net = gen.make_network(2, [([(0, 1), (1, 1)], [])]); x0 = [x, x]; c = 0.2
        a, nu, g = c * x * x, -1, 2.0
    else:
        net = gen.make_network(1, [([(0, 2)], [])]); x0 = [x]; c = 1.0
        a, nu, g = c * x * (x - 1) / 2, -2, 2.0 + 1.0 / (x - 1)
    b = max(eps * x / g, 1.0)
    mu, sig = nu * a, nu * nu * a
    tau = min(b / abs(mu), b * b / sig)
    lam = a * tau
    runs = 200000
    out, st, _ = _run(net, [c], x0, [0.0, 1000.0], seed=34, runs=runs, eps=eps, n_c=0,
                      ssa_factor=0.0, max_steps=1)
    k = np.arange(0, 60)
    pk = sst.poisson.pmf(k, lam)
    ok = x + nu * k >= 0
    pmf = {}
    for kk, p, good in zip(k, pk, ok):
        v = x + nu * kk if good else x
        pmf[int(v)] = pmf.get(int(v), 0.0) + float(p)
    assert chi2_pvalue(out[1, 0], pmf) > 1e-3
    assert np.array_equal(st[:, 0] + st[:, 2], np.ones(runs, dtype=np.uint64))


def test_rejection_halves_tau():
    # A -> 0 from x = 6 with eps = 0.9 (b = eps x, so lam = b = 5.4): a proposal
    # k > 6 is rejected and the retry uses tau'/2 (lam 2.7).  max_steps = 2 stops
    # the run after two attempts; the exact law of the result follows.
    eps, x0 = 0.9, 6
    net = gen.decay_network()
    runs = 200000
    out, st, _ = _run(net, [1.0], [x0], [0.0, 1000.0], seed=35, runs=runs, eps=eps, n_c=0,
                      ssa_factor=0.0, max_steps=2)
    ks = np.arange(0, 80)

    def leap(x, lam):  # distribution after one attempt from x (rejections keep x)
        d = {}
        for k, p in zip(ks, sst.poisson.pmf(ks, lam)):
            y = x - k if k <= x else x
            d[y] = d.get(y, 0.0) + p
        return d

    law = {}
    lam1 = max(eps * x0, 1.0)
    for k, p in zip(ks, sst.poisson.pmf(ks, lam1)):
        if k <= x0:          # accepted: a fresh decision from x0 - k
            x1 = x0 - k
            nxt = leap(x1, max(eps * x1, 1.0)) if x1 > 0 else {0: 1.0}
        else:                # rejected: retry with half the leap
            nxt = leap(x0, lam1 / 2)
        for y, q in nxt.items():
            law[y] = law.get(y, 0.0) + p * q
    assert chi2_pvalue(out[1, 0], law) > 1e-3


def test_critical_threshold_is_strict():
    # L_j = x for A -> 0; the reaction is critical iff L_j < n_c.  From x = 10
    # with n_c = 10 it is not critical (a Poisson leap); from x = 9 it is, and
    # the single attempt fires it exactly once.
    net = gen.decay_network()
    runs = 20000
    out, _, _ = _run(net, [1.0], [9], [0.0, 1000.0], seed=36, runs=runs, eps=0.5, n_c=10,
                     ssa_factor=0.0, max_steps=1)
    assert np.all(out[1, 0] == 8)
    out, _, _ = _run(net, [1.0], [10], [0.0, 1000.0], seed=36, runs=runs, eps=0.5, n_c=10,
                     ssa_factor=0.0, max_steps=1)
    assert len(np.unique(out[1, 0])) > 5


def test_clipped_leap_lands_exactly_on_the_sample_time():
    # 0.299 + (0.971 - 0.299) rounds below 0.971; a leap clipped to a sample
    # time must set t to that time, so the source takes exactly one leap per
    # sample interval and no extra sliver of a leap.
    net = gen.source_network()
    out, st, _ = _run(net, [2.0], [0], [0.0, 0.299, 0.971], seed=37, runs=100)
    assert 0.299 + (0.971 - 0.299) < 0.971
    assert np.all(st[:, 0] == 2)


def test_single_leap_signed_drift():
    # A <-> B with equal fluxes: mu_A = -a1 + a2 = 0, so tau' comes from
    # sigma^2 = a1 + a2 alone (an unsigned drift would halve tau').  One attempt:
    # x_A' = 60 - k1 + k2 with k1, k2 ~ Poisson(a tau').
    net = gen.isomerization_network()
    eps, x = 0.03, 60
    b = max(eps * x, 1.0)
    a = 1.0 * x
    tau = b * b / (2 * a)
    lam = a * tau
    runs = 200000
    out, st, _ = _run(net, [1.0, 1.0], [x, x], [0.0, 1000.0], seed=38, runs=runs, eps=eps,
                      n_c=0, ssa_factor=0.0, max_steps=1)
    assert np.all(st[:, 2] == 0)
    k = np.arange(0, 40)
    p = sst.poisson.pmf(k, lam)
    law = {}
    for k1, p1 in zip(k, p):
        for k2, p2 in zip(k, p):
            law[int(x - k1 + k2)] = law.get(int(x - k1 + k2), 0.0) + p1 * p2
    assert chi2_pvalue(out[1, 0], law) > 1e-3


def test_ssa_bursts_then_leaps():
    # birth-death k1 = 1000, k2 = 1 from x = 0: while x is small tau' is below
    # 10/a0 and the run takes whole bursts of 100 exact events; once x is a few
    # hundred it leaps.  SSA counts are therefore positive multiples of the burst.
    net = gen.birth_death_network()
    out, st, _ = _run(net, [1000.0, 1.0], [0], gen.sample_times(5.0, 6), seed=39, runs=500)
    assert np.all(st[:, 1] > 0) and np.all(st[:, 0] > 0)
    assert np.all(st[:, 1] % 100 == 0)
    out2, st2, _ = _run(net, [1000.0, 1.0], [0], gen.sample_times(5.0, 6), seed=39, runs=500,
                        ssa_burst=37)
    assert np.all(st2[:, 1] % 37 == 0) and np.all(st2[:, 1] > 0)
