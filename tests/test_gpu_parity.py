"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 mode shares the oracle's counter-based random streams and its rounding
order, so trajectories are compared element by element: at least 99.9% of them
must be identical (samples and step statistics), and no count may be negative.
The only licensed source of a mismatch is a last-bit difference between the
host and device libm in exp/log/lgamma.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1309_7695_amd import gen, rn

pytestmark = pytest.mark.gpu

MIN_IDENTICAL = 0.999


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.dirname(rn.LIB_PATH).endswith("paper_1309_7695_amd")
    rn.lib()
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(out, st, ref, rst, what, min_identical=MIN_IDENTICAL):
    assert out.shape == ref.shape and st.shape == rst.shape
    assert out.min() >= 0, f"{what}: negative count"
    same = np.all(out == ref, axis=(0, 1)) & np.all(st == rst, axis=1)
    frac = same.mean()
    _say(f"{what}: {same.sum()}/{same.size} trajectories identical")
    assert frac >= min_identical, f"{what}: only {frac:.5f} identical"
    return same


def _both(w, seed, threads=8, **kw):
    _say(f"case {w.name}: T={w.n_traj} seed={seed} {kw}")
    out, st = rn.run(w.net, w.rates, w.x0, w.times, seed=seed, **kw)
    ref, rst, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=seed, threads=threads, **kw)
    return out, st, ref, rst


def _tiny(net, rates, x0, times, runs):
    rates = np.repeat(np.asarray(rates, float)[:, None], runs, axis=1)
    return gen.Workload(net.name, net, rates, np.asarray(x0, np.int32), np.asarray(times, float))


def test_enzyme_workload_full():
    w = gen.enzyme_workload()
    out, st, ref, rst = _both(w, seed=1)
    _compare(out, st, ref, rst, "enzyme 4x3, 1024 trajectories")
    assert np.all(out[:, 0] + out[:, 2] == 100)


def test_synthetic_network_ragged_subset():
    # the 50-species, 100-reaction network: 300 trajectories = 4 full waves and a
    # ragged tail
    w = gen.synthetic_workload(n_traj=300)
    out, st, ref, rst = _both(w, seed=2)
    _compare(out, st, ref, rst, "synthetic 50x100, 300 trajectories")


def test_synthetic_full_size_sampled():
    # the full 65,536-trajectory sweep in its production launch shape; the oracle
    # checks a sample of trajectory ids one by one
    import torch
    w = gen.synthetic_workload()
    T = w.n_traj
    _say(f"case synthetic 50x100 full: T={T}")
    dev = torch.device("cuda:0")
    net = rn.Network(w.net)
    r = torch.from_numpy(w.rates).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o = torch.empty((len(w.times), w.net.n_species, T), dtype=torch.int32, device=dev)
    s = torch.empty((T, 4), dtype=torch.int64, device=dev)
    rn.sweep(net, r, x, tm, o, s, seed=2)
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    ids = np.unique(np.concatenate([[0, 63, 64, 255, 256, T - 1],
                                    rng.integers(0, T, size=58)]))
    idt = torch.from_numpy(ids).to(dev)
    out = o.index_select(2, idt).cpu().numpy()
    st = s.index_select(0, idt).cpu().numpy().view(np.uint64)
    assert int(o.min().item()) >= 0
    ref = np.zeros_like(out)
    rst = np.zeros_like(st)
    for k, i in enumerate(ids):
        a, b, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=2, traj_range=(int(i), int(i) + 1))
        ref[:, :, k] = a[:, :, 0]
        rst[k] = b[0]
    same = np.all(out == ref, axis=(0, 1)) & np.all(st == rst, axis=1)
    _say(f"full-size sample: {same.sum()}/{len(ids)} identical")
    assert same.sum() >= len(ids) - 1


def test_stiff_network_subset():
    w = gen.stiff_workload(n_traj=200)
    out, st, ref, rst = _both(w, seed=4)
    _compare(out, st, ref, rst, "stiff 30x80, 200 trajectories")


@pytest.mark.parametrize("form", ["0", "1"])
def test_large_network(monkeypatch, form):
    # 500 reactions, 250 species: the largest network of the uneven batch, on
    # the lane-per-trajectory (RN_WSWEEP=0) and the wave-per-trajectory form
    monkeypatch.setenv("RN_WSWEEP", form)
    net = gen.random_network(3001, 250, 500)
    rng = np.random.default_rng(5)
    T = 96
    rates = gen.log_uniform(rng, 1e-4, 1.0, 500)[:, None] * gen.log_uniform(rng, 0.1, 10, (500, T))
    x0 = rng.integers(0, 1001, size=250).astype(np.int32)
    w = gen.Workload("random 250x500", net, np.ascontiguousarray(rates), x0,
                     gen.sample_times(2.0, 11))
    out, st, ref, rst = _both(w, seed=7)
    _compare(out, st, ref, rst, "random 250x500, 96 trajectories")


def test_per_trajectory_initial_counts_and_offset():
    w = gen.synthetic_workload(n_traj=150, n_species=12, n_reactions=24, t_end=10.0,
                               n_samples=21)
    rng = np.random.default_rng(3)
    x0 = rng.integers(0, 300, size=(12, 150)).astype(np.int32)
    w2 = gen.Workload("perx0", w.net, w.rates, x0, w.times)
    out, st, ref, rst = _both(w2, seed=9)
    _compare(out, st, ref, rst, "per-trajectory x0")


def test_trajectory_range_reproduces_slice():
    import torch
    w = gen.synthetic_workload(n_traj=256, n_species=10, n_reactions=20, t_end=5.0,
                               n_samples=11)
    dev = torch.device("cuda:0")
    full, sfull = rn.run(w.net, w.rates, w.x0, w.times, seed=5)
    net = rn.Network(w.net)
    a, b = 70, 201
    r = torch.from_numpy(np.ascontiguousarray(w.rates[:, a:b])).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o = torch.empty((11, 10, b - a), dtype=torch.int32, device=dev)
    s = torch.empty((b - a, 4), dtype=torch.int64, device=dev)
    rn.sweep(net, r, x, tm, o, s, seed=5, traj_offset=a)
    torch.cuda.synchronize()
    assert np.array_equal(o.cpu().numpy(), full[:, :, a:b])
    assert np.array_equal(s.cpu().numpy().view(np.uint64), sfull[a:b])


def test_deterministic_repeat():
    w = gen.synthetic_workload(n_traj=128, n_species=10, n_reactions=20, t_end=5.0, n_samples=6)
    o1, s1 = rn.run(w.net, w.rates, w.x0, w.times, seed=11)
    o2, s2 = rn.run(w.net, w.rates, w.x0, w.times, seed=11)
    assert np.array_equal(o1, o2) and np.array_equal(s1, s2)


@pytest.mark.parametrize("case", ["source", "catalytic", "decay80", "allcrit", "ssa", "reject",
                                  "absorb", "maxsteps", "overflow", "single_sample", "dimer",
                                  "cle_decay", "cle_birth_death"])
def test_small_cases_bitwise(case):
    kw = {}
    if case == "source":
        w = _tiny(gen.source_network(), [40.0], [0], [0.0, 0.5, 1.0, 2.0], 1000)
    elif case == "catalytic":
        w = _tiny(gen.catalytic_network(), [0.7], [20, 0], [0.0, 0.25, 1.0], 1000)
    elif case == "decay80":
        w = _tiny(gen.decay_network(), [1.0], [100000], gen.sample_times(2.0, 21), 500)
    elif case == "allcrit":
        w = _tiny(gen.enzyme_network(), [0.3, 0.5, 0.7], [2, 5, 0, 0], [0.0, 5.0], 1000)
    elif case == "ssa":
        w = _tiny(gen.isomerization_network(), [1.0, 0.5], [10, 0], [0.0, 0.2, 1.0, 3.0], 1000)
        kw["method"] = "ssa"
    elif case == "reject":
        w = _tiny(gen.reversible_dimer_network(), [0.5, 5.0], [60, 20],
                  gen.sample_times(5.0, 11), 1000)
        kw.update(eps=0.9, n_c=0, ssa_factor=0.0)
    elif case == "absorb":
        w = _tiny(gen.decay_network(), [5.0], [3], gen.sample_times(10.0, 11), 200)
    elif case == "maxsteps":
        w = _tiny(gen.birth_death_network(), [10.0, 0.1], [0], gen.sample_times(100.0, 11), 200)
        kw.update(max_steps=7, method="ssa")
    elif case == "overflow":
        w = _tiny(gen.source_network(), [1e12], [0], [0.0, 1.0], 64)
    elif case == "single_sample":
        w = _tiny(gen.birth_death_network(), [5.0, 1.0], [3], [2.0], 100)
    elif case == "cle_decay":
        w = _tiny(gen.decay_network(), [1.0], [100000], gen.sample_times(2.0, 21), 500)
        kw["cle_threshold"] = 100.0
    elif case == "cle_birth_death":
        w = _tiny(gen.birth_death_network(), [2000.0, 1.0], [0], gen.sample_times(5.0, 11), 500)
        kw["cle_threshold"] = 50.0
    else:
        w = _tiny(gen.reversible_dimer_network(), [0.02, 1.0], [500, 100],
                  gen.sample_times(3.0, 7), 300)
    out, st, ref, rst = _both(w, seed=31, **kw)
    same = _compare(out, st, ref, rst, case,
                    min_identical=0.999 if case.startswith("cle") else 1.0)
    if case == "reject":
        assert st[:, 2].sum() > 0
    if case == "overflow":
        assert np.all(st[:, 3] == rn.ST_OVERFLOW)
    if case == "absorb":
        assert np.all(st[:, 3] == rn.ST_ABSORBED)
    if case == "maxsteps":
        assert np.all(st[:, 3] == rn.ST_MAXSTEPS)
    if case in ("decay80", "cle_decay"):
        assert np.all(st[:, 0] == 80)
    if not case.startswith("cle"):
        assert same.all()


def test_empty_sweep_is_a_noop():
    import torch
    dev = torch.device("cuda:0")
    net = rn.Network(gen.decay_network())
    r = torch.zeros((1, 1), dtype=torch.float64, device=dev)
    x = torch.zeros(1, dtype=torch.int32, device=dev)
    tm = torch.zeros(1, dtype=torch.float64, device=dev)
    o = torch.full((1, 1, 1), -7, dtype=torch.int32, device=dev)
    s = torch.empty((0, 4), dtype=torch.int64, device=dev)
    rn.sweep(net, r, x, tm, o, s, seed=1)
    torch.cuda.synchronize()
    assert int(o.item()) == -7


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_network_compiled_kernel_matches_generic(monkeypatch, precision):
    # the kernel compiled for one network and the generic kernel evaluate the
    # same operations in the same order: identical trajectories in either
    # precision (the 50x100 network, 300 trajectories with a ragged last wave)
    w = gen.synthetic_workload(n_traj=300)
    net = rn.Network(w.net)
    _say(f"case network-compiled vs generic {precision}")
    assert rn.sweep_kernel_kind(net, w.n_traj, precision) == "network"
    a, sa = rn.run(net, w.rates, w.x0, w.times, seed=21, precision=precision)
    monkeypatch.setenv("RN_JIT", "0")
    monkeypatch.setenv("RN_WSWEEP", "0")
    assert rn.sweep_kernel_kind(net, w.n_traj, precision) == "generic"
    b, sb = rn.run(net, w.rates, w.x0, w.times, seed=21, precision=precision)
    same = np.all(a == b, axis=(0, 1)) & np.all(sa == sb, axis=1)
    _say(f"  {same.sum()}/{same.size} identical")
    assert same.all()


def test_large_network_uses_generic_kernel(monkeypatch):
    # no compiled kernel; few trajectories: one wave each, unless RN_WSWEEP=0
    net = rn.Network(gen.random_network(3001, 250, 500))
    monkeypatch.delenv("RN_WSWEEP", raising=False)
    assert rn.sweep_kernel_kind(net, 96) == "wave"
    monkeypatch.setenv("RN_WSWEEP", "0")
    assert rn.sweep_kernel_kind(net, 96) == "generic"
