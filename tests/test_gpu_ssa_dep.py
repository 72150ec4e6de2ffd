"""Exact SSA (RN_METHOD_SSA) on the dependency-graph kernel: propensities are
kept between events and only those whose reactants an event changed are
recomputed; a0 and the pick still use the running sums in index order.  Its
trajectories must be the oracle's direct-method trajectories bit for bit, and
identical to those of the general network-compiled kernel (RN_SSA_KERNEL=full),
in both precisions."""
import os

import numpy as np
import pytest

import oracle
from paper_1309_7695_amd import gen, rn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rn.lib()


def _gpu(w, seed, kernel, precision="fp64", **kw):
    old = os.environ.get("RN_SSA_KERNEL")
    os.environ["RN_SSA_KERNEL"] = kernel
    try:
        return rn.run(w.net, w.rates, w.x0, w.times, seed=seed, method="ssa",
                      precision=precision, **kw)
    finally:
        if old is None:
            del os.environ["RN_SSA_KERNEL"]
        else:
            os.environ["RN_SSA_KERNEL"] = old


def _case(w, seed, **kw):
    print(f"case ssa-dep {w.name}: T={w.n_traj}", flush=True)
    out, st = _gpu(w, seed, "dep", **kw)
    full, fst = _gpu(w, seed, "full", **kw)
    assert np.array_equal(out, full) and np.array_equal(st, fst), "dependency vs general kernel"
    ref, rst, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=seed, method="ssa", threads=16,
                             **kw)
    same = np.all(out == ref, axis=(0, 1)) & np.all(st == rst, axis=1)
    print(f"  identical to the oracle: {same.mean():.4f}; events {int(st[:, 1].sum())}",
          flush=True)
    assert same.mean() >= 0.999
    assert out.min() >= 0
    return out, st


def test_ssa_dep_enzyme():
    _case(gen.enzyme_workload(), 21)


def test_ssa_dep_synthetic():
    _case(gen.synthetic_workload(n_traj=300, t_end=0.5, n_samples=11), 22)


def test_ssa_dep_synthetic_full_workgroups():
    # enough trajectories for 256-lane workgroups (four waves sharing LDS)
    w = gen.synthetic_workload(n_traj=65536, t_end=0.02, n_samples=3)
    out, st = _gpu(w, 23, "dep")
    full, fst = _gpu(w, 23, "full")
    assert np.array_equal(out, full) and np.array_equal(st, fst)
    ids = np.linspace(0, w.n_traj - 1, 16).astype(int)
    for t in ids:
        ref, rst, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=23, method="ssa",
                                 traj_range=(int(t), int(t) + 1))
        assert np.array_equal(out[:, :, t], ref[:, :, 0]) and np.array_equal(st[t], rst[0])


def test_ssa_dep_stiff():
    _case(gen.stiff_workload(n_traj=200), 24)


def test_ssa_dep_status_rules():
    # max_steps mid-run and an absorbing network
    w = gen.enzyme_workload(n_traj=100)
    _case(w, 25, max_steps=57)
    d = gen.decay_network()
    rates = np.full((1, 64), 2.0)
    times = gen.sample_times(5.0, 6)
    wd = gen.Workload(name="decay", net=d, rates=rates, x0=np.array([5], np.int32), times=times)
    out, st = _case(wd, 26)
    assert np.all(st[:, 3] & rn.ST_ABSORBED)


def test_ssa_dep_fp32_equals_general_kernel():
    w = gen.synthetic_workload(n_traj=500, t_end=0.5, n_samples=11)
    out, st = _gpu(w, 27, "dep", precision="fp32")
    full, fst = _gpu(w, 27, "full", precision="fp32")
    assert np.array_equal(out, full) and np.array_equal(st, fst)
