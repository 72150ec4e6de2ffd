"""Pins of the oracle's exact-SSA path against the chemical master equation and
closed forms (the law of X(t): paper, Methods section)."""
import numpy as np
import pytest
from scipy import stats as sst

import oracle
from paper_1309_7695_amd import gen
from tests import cme
from tests.stats_util import chi2_pvalue, z_mean, z_var

RUNS = 100000


def _ssa(net, rates_nominal, x0, times, seed, runs=RUNS, method="ssa", **kw):
    rates = np.repeat(np.asarray(rates_nominal, dtype=float)[:, None], runs, axis=1)
    out, st, _ = oracle.run(net, rates, np.asarray(x0, dtype=np.int32), np.asarray(times, float),
                            seed=seed, method=method, threads=8, **kw)
    return out, st


def _check_cme(net, rates, x0, times, out, cap=None, species=(0,)):
    for s, t in enumerate(times):
        if t == 0:
            continue
        dist = cme.distribution(net, rates, x0, t, cap=cap)
        for sp in species:
            pmf = cme.marginal(dist, sp)
            p = chi2_pvalue(out[s, sp], pmf)
            assert p > 1e-3, (net.name, t, sp, p)


def test_decay_binomial():
    net = gen.decay_network()
    times = [0.0, 0.3, 1.0, 2.0]
    out, st = _ssa(net, [1.0], [8], times, seed=5)
    for s, t in enumerate(times):
        p = np.exp(-t)
        pmf = {k: float(sst.binom.pmf(k, 8, p)) for k in range(9)}
        assert chi2_pvalue(out[s, 0], pmf) > 1e-3
        assert z_mean(out[s, 0], 8 * p) < 4 if t > 0 else np.all(out[s, 0] == 8)
    # every run ends absorbed once all molecules decayed, or was still alive at t=2
    assert np.all((st[:, 3] == 0) | (st[:, 3] == oracle.ST_ABSORBED))


def test_birth_death_closed_form():
    net = gen.birth_death_network()
    k1, k2, x0 = 5.0, 1.0, 10
    times = [0.0, 0.5, 1.0, 3.0]
    out, _ = _ssa(net, [k1, k2], [x0], times, seed=6)
    for s, t in enumerate(times[1:], start=1):
        p = np.exp(-k2 * t)
        m = x0 * p + (k1 / k2) * (1 - p)
        v = x0 * p * (1 - p) + (k1 / k2) * (1 - p)
        assert z_mean(out[s, 0], m) < 4
        assert z_var(out[s, 0], v) < 4
        # X = Bin(x0, p) + Poi(k1/k2 (1-p))
        kmax = 60
        b = sst.binom.pmf(np.arange(kmax), x0, p)
        q = sst.poisson.pmf(np.arange(kmax), (k1 / k2) * (1 - p))
        pmf = np.convolve(b, q)[:kmax]
        assert chi2_pvalue(out[s, 0], pmf) > 1e-3


def test_birth_death_stationary_poisson():
    net = gen.birth_death_network()
    out, _ = _ssa(net, [4.0, 2.0], [0], [0.0, 20.0], seed=7, runs=50000)
    pmf = sst.poisson.pmf(np.arange(40), 2.0)
    assert chi2_pvalue(out[1, 0], pmf) > 1e-3


def test_isomerization_cme():
    net = gen.isomerization_network()
    rates, x0, times = [1.0, 0.5], [10, 0], [0.0, 0.2, 1.0, 3.0]
    out, _ = _ssa(net, rates, x0, times, seed=8)
    _check_cme(net, rates, x0, times, out)
    assert np.all(out[:, 0] + out[:, 1] == 10)


def test_dimerization_cme_pins_binomial_two():
    # 2A -> B with propensity c*x(x-1)/2: a factor-2 slip fails this test
    net = gen.dimerization_network()
    rates, x0, times = [0.1], [12, 0], [0.0, 0.2, 0.5, 2.0]
    out, _ = _ssa(net, rates, x0, times, seed=9)
    _check_cme(net, rates, x0, times, out, species=(0, 1))
    assert np.all(out[:, 0] + 2 * out[:, 1] == 12)


def test_enzyme_small_cme():
    net = gen.enzyme_network()
    rates, x0, times = [0.3, 0.5, 0.7], [2, 5, 0, 0], [0.0, 0.5, 2.0, 6.0]
    out, _ = _ssa(net, rates, x0, times, seed=10)
    _check_cme(net, rates, x0, times, out, species=(0, 1, 3))


@pytest.mark.parametrize("name,rates,x0,times", [
    ("enzyme", [0.3, 0.5, 0.7], [2, 5, 0, 0], [0.0, 0.5, 2.0, 6.0]),
    ("isomerization", [1.0, 0.5], [8, 0], [0.0, 0.2, 1.0, 3.0]),
])
def test_tauleap_all_critical_matches_cme(name, rates, x0, times):
    # every count stays below n_c = 10, so every reaction is critical and each
    # leap fires at most one reaction: the leap path must reproduce the CME law
    net = getattr(gen, name + "_network")()
    out, st = _ssa(net, rates, x0, times, seed=12, method="tauleap")
    assert st[:, 1].sum() == 0  # tau' is infinite: never an SSA burst
    _check_cme(net, rates, x0, times, out, species=(0, 1))
