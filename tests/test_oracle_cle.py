"""Pins of the Chemical-Langevin (Gaussian increment) leap option."""
import numpy as np
import pytest
from scipy import stats as sst

import oracle
from paper_1309_7695_amd import gen
from tests.stats_util import chi2_pvalue, z_mean, z_var


@pytest.mark.parametrize("lam", [50.0, 1e3, 1e5])
def test_cle_count_is_rounded_gaussian(lam):
    n = 200000
    k = oracle.cle_many(lam, seed=5, n=n, j=7)
    assert k.min() >= 0
    sd = np.sqrt(lam)
    lo, hi = int(lam - 7 * sd), int(lam + 7 * sd) + 1
    ks = np.arange(max(lo, 0), hi + 1)
    pmf = sst.norm.cdf((ks + 0.5 - lam) / sd) - sst.norm.cdf((ks - 0.5 - lam) / sd)
    assert chi2_pvalue(k, dict(zip(ks.tolist(), pmf.tolist()))) > 1e-3
    assert z_mean(k, lam) < 4.5
    assert z_var(k, lam + 1.0 / 12.0) < 4.5


def test_cle_floors_at_zero():
    k = oracle.cle_many(10.0, seed=1, n=200000)
    assert k.min() >= 0


def test_cle_decay_leaps_match_poisson_moments():
    # same deterministic 80-leap sequence as the Poisson pin; Gaussian increments
    # with the Poisson mean and variance give the same first two moments
    net = gen.decay_network()
    times = gen.sample_times(2.0, 21)
    runs = 20000
    rates = np.full((1, runs), 1.0)
    out, st, _ = oracle.run(net, rates, np.array([100000], np.int32), times, seed=3, threads=8,
                            cle_threshold=100.0)
    assert np.all(st[:, 0] == 80)
    m, v = 1e5, 0.0
    for s in range(1, 21):
        for tau in [0.03, 0.03, 0.03, times[s] - (times[s - 1] + 0.09)]:
            v = (1 - tau) ** 2 * v + tau * m + 1.0 / 12.0
            m = (1 - tau) * m
        assert z_mean(out[s, 0], m) < 4.5
        assert z_var(out[s, 0], v) < 4.5


def test_cle_off_is_plain_poisson_bitwise():
    w = gen.synthetic_workload(n_traj=32, n_species=10, n_reactions=20, t_end=5.0, n_samples=6)
    a, sa, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=4)
    b, sb, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=4, cle_threshold=0.0)
    assert np.array_equal(a, b) and np.array_equal(sa, sb)


def test_cle_threshold_must_exceed_poisson_inversion_range():
    net = gen.decay_network()
    with pytest.raises(RuntimeError):
        oracle.run(net, np.ones((1, 2)), np.array([5], np.int32), [0.0, 1.0], seed=1,
                   cle_threshold=5.0)
