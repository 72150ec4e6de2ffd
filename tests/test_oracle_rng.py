"""Pins of the oracle's random-number layer (Philox4x32-10, U53, Poisson)."""
import os

import numpy as np
import pytest
from scipy import stats as sst

import oracle
from tests.stats_util import chi2_pvalue, z_mean, z_var

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(w, 16) for w in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = [int(w) for w in oracle.philox4x32_10(ctr, key)]
        assert got == want, (ctr, key, [hex(g) for g in got])


def test_philox_is_a_bijection_on_a_sample():
    rng = np.random.default_rng(0)
    seen = set()
    for _ in range(2000):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        out = tuple(int(w) for w in oracle.philox4x32_10(ctr, [123, 456]))
        assert out not in seen
        seen.add(out)


def test_u53_edges():
    assert oracle.u53(0, 0) == 0.0
    assert oracle.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    assert oracle.u53(0, 0x800) == 2.0**-53       # lowest kept bit
    assert oracle.u53(0, 0x7FF) == 0.0           # discarded bits
    assert oracle.u53(0x80000000, 0) == 0.5


def test_philox_words_uniform_bytes():
    # byte chi-square over 20000 blocks of the event stream
    words = []
    for t in range(20000):
        words.extend(int(w) for w in oracle.philox4x32_10([t, 0, 0, 0], [7, 0]))
    b = np.frombuffer(np.asarray(words, dtype=np.uint32).tobytes(), dtype=np.uint8)
    cnt = np.bincount(b, minlength=256)
    p = sst.chisquare(cnt).pvalue
    assert p > 1e-4


@pytest.mark.parametrize("lam", [1e-3, 0.5, 3.0, 9.999, 10.0, 30.0, 1e3, 1e6])
def test_poisson_distribution(lam):
    n = 200000
    v = oracle.poisson_many(lam, seed=11, n=n, j=3)
    assert v.min() >= 0
    assert z_mean(v, lam) < 4.5
    assert z_var(v, lam) < 4.5
    lo = int(max(0, sst.poisson.ppf(1e-9, lam)))
    hi = int(sst.poisson.ppf(1 - 1e-9, lam)) + 1
    ks = np.arange(lo, hi + 1)
    pmf = {int(k): float(sst.poisson.pmf(k, lam)) for k in ks}
    assert chi2_pvalue(v, pmf) > 1e-3


def test_poisson_degenerate():
    assert oracle.poisson(0.0, 1, 0, 0, 0) == 0
    assert oracle.poisson(-1.0, 1, 0, 0, 0) == 0
    assert oracle.poisson(float("nan"), 1, 0, 0, 0) == 0


def test_poisson_pairs_share_one_block_but_not_one_uniform():
    # reactions 2p and 2p+1 take the two halves of one block: different uniforms
    a = oracle.poisson_many(5.0, seed=3, n=50000, j=4)
    b = oracle.poisson_many(5.0, seed=3, n=50000, j=5)
    assert not np.array_equal(a, b)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.03


def test_poisson_huge_mean_is_clamped():
    v = oracle.poisson_many(1e13, seed=1, n=10)
    assert np.all(v == 2**31)
