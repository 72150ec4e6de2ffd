"""Pins for the two decisions of the oracle whose ties no trajectory statistic
can see, checked against their published definitions in exact arithmetic.

* The direct method's selection (Gillespie 1977): with propensities a_j and
  r = u * a0, the reaction fired is the smallest j with a_0 + ... + a_j > r.
  When r lands exactly on a partial sum a_0 + ... + a_k, the next reaction with
  a positive propensity fires, never reaction k.
* The critical race (Cao, Gillespie and Petzold 2006): a critical reaction fires
  when its waiting time tau'' does not exceed the leap bound tau'; on equality
  it fires.  The sample-time cap (tau'' also no later than the next sample
  time) is this project's reading for sampled sweeps.

Propensities are multiples of 1/8 below 64, so every partial sum is exact in
FP64 and the exact-rational reference applies bit for bit."""
from fractions import Fraction

import numpy as np

import oracle


def _textbook_pick(a, r, allowed=None):
    # smallest allowed j whose exact running sum exceeds r; None if there is none
    acc = Fraction(0)
    for j, v in enumerate(a):
        if allowed is not None and not allowed[j]:
            continue
        acc += Fraction(v)
        if Fraction(r) < acc:
            return j
    return None


def test_pick_on_exact_partial_sums():
    a = [0.5, 0.25, 0.0, 0.25]
    # r on each partial sum: 0.5 -> reaction 1, 0.75 -> reaction 3 (2 has a = 0)
    assert oracle.pick_index(a, 0.5) == 1
    assert oracle.pick_index(a, 0.75) == 3
    assert oracle.pick_index(a, 0.0) == 0
    # zero propensities never fire, even at r = 0
    assert oracle.pick_index([0.0, 0.0, 2.0, 0.0], 0.0) == 2


def test_pick_matches_the_definition_on_random_ties():
    rng = np.random.default_rng(11)
    for _ in range(400):
        m = int(rng.integers(1, 12))
        a = (rng.integers(0, 64 * 8, size=m) / 8.0) * (rng.random(m) < 0.8)
        if a.sum() == 0:
            continue
        partial = np.cumsum(a)
        allowed = (rng.random(m) < 0.7).astype(np.int32)
        # every partial sum (a tie) and a point strictly inside every interval
        # (below a0: r = u * a0 with u < 1)
        rs = [r for r in list(partial[:-1]) + list(partial - a / 2) + [0.0] if r < partial[-1]]
        for r in rs:
            want = _textbook_pick(a, r)
            assert want is not None
            assert oracle.pick_index(a, r) == want, (a, r)
            want_al = _textbook_pick(a, r, allowed)
            if want_al is not None:
                assert oracle.pick_index(a, r, allowed) == want_al, (a, r, allowed)


def test_pick_when_rounding_leaves_no_reaction():
    # r >= a0 cannot happen in exact arithmetic (u < 1); the oracle's reading
    # then fires the last reaction with a positive propensity
    a = [1.0, 2.0, 0.0]
    assert oracle.pick_index(a, 3.0) == 1
    assert oracle.pick_index(a, 5.0) == 1
    assert oracle.pick_index([0.0, 0.0], 0.0) == -1
    assert oracle.pick_index(a, 3.0, [1, 0, 1]) == 0


def test_critical_race_ties():
    one = 1.0
    above = np.nextafter(one, 2.0)
    below = np.nextafter(one, 0.0)
    # tau'' == tau' fires; one ulp later it does not
    assert oracle.critical_fires(one, one, 10.0) == 1
    assert oracle.critical_fires(above, one, 10.0) == 0
    assert oracle.critical_fires(below, one, 10.0) == 1
    # the sample-time cap: tau'' equal to the time left fires, one ulp more does not
    assert oracle.critical_fires(one, 10.0, one) == 1
    assert oracle.critical_fires(above, 10.0, one) == 0
    # no critical reaction (tau'' infinite) never fires
    assert oracle.critical_fires(np.inf, 10.0, 10.0) == 0
