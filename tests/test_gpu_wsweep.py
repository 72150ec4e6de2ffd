"""The one-wave-per-trajectory sweep (rn_wsweep.hip): lanes hold reactions and
species, and the sums whose value depends on their order (a0, the SSA pick, a0c
and the critical pick) walk the reactions in index order.  In FP64 its
trajectories must be the oracle's bit for bit (the rule of test_gpu_parity.py);
in both precisions they must equal, bit for bit, those of the
lane-per-trajectory generic kernel on the same inputs.  RN_JIT=0 keeps the
network-compiled kernel out; RN_WSWEEP picks the generic form."""
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
    rn.lib()


@pytest.fixture
def generic(monkeypatch):
    monkeypatch.setenv("RN_JIT", "0")

    def run(w, seed, form, **kw):
        monkeypatch.setenv("RN_WSWEEP", "1" if form == "wave" else "0")
        net = rn.Network(w.net)
        kind = rn.sweep_kernel_kind(net, w.n_traj, kw.get("precision", "fp64"))
        assert kind == form, (kind, form)
        return rn.run(net, w.rates, w.x0, w.times, seed=seed, **kw)

    return run


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _vs_oracle(out, st, w, seed, what, **kw):
    ref, rst, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=seed, threads=16, **kw)
    assert out.min() >= 0, f"{what}: negative count"
    same = np.all(out == ref, axis=(0, 1)) & np.all(st == rst, axis=1)
    _say(f"{what}: {same.sum()}/{same.size} trajectories identical to the oracle")
    assert same.mean() >= MIN_IDENTICAL


def _vs_lanes(generic, w, seed, what, **kw):
    out, st = generic(w, seed, "wave", **kw)
    lo, lst = generic(w, seed, "generic", **kw)
    same = np.all(out == lo, axis=(0, 1)) & np.all(st == lst, axis=1)
    _say(f"{what}: {same.sum()}/{same.size} identical to the lane-per-trajectory kernel; "
         f"steps {int(st[:, 0].sum() + st[:, 1].sum())}")
    assert same.all()
    return out, st


@pytest.mark.parametrize("name", ["enzyme", "synthetic", "stiff", "wide"])
def test_wave_kernel_matches_oracle_and_lanes(generic, name):
    # K = 1 (3 reactions), 2 (100), 2 (80) and 4 (180) reaction registers per lane
    w = {"enzyme": lambda: gen.enzyme_workload(),
         "synthetic": lambda: gen.synthetic_workload(n_traj=300, t_end=10.0, n_samples=21),
         "stiff": lambda: gen.stiff_workload(n_traj=200),
         "wide": lambda: gen.synthetic_workload(n_traj=150, seed=3200, n_species=90,
                                                n_reactions=180, t_end=2.0, n_samples=9)}[name]()
    _say(f"case wave {w.name}: T={w.n_traj} N={w.net.n_species} M={w.net.n_reactions}")
    out, st = _vs_lanes(generic, w, 31, f"wave {w.name}")
    _vs_oracle(out, st, w, 31, f"wave {w.name}")


def test_wave_kernel_largest_network(monkeypatch):
    # 250 species, 500 reactions (K = 8): the default policy picks the wave form
    # for 96 trajectories; the oracle decides
    monkeypatch.delenv("RN_WSWEEP", raising=False)
    net = gen.random_network(3001, 250, 500)
    rng = np.random.default_rng(5)
    T = 96
    rates = gen.log_uniform(rng, 1e-4, 1.0, 500)[:, None] * gen.log_uniform(rng, 0.1, 10, (500, T))
    x0 = rng.integers(0, 1001, size=250).astype(np.int32)
    w = gen.Workload("random 250x500", net, np.ascontiguousarray(rates), x0,
                     gen.sample_times(2.0, 11))
    h = rn.Network(w.net)
    assert rn.sweep_kernel_kind(h, T) == "wave"
    out, st = rn.run(h, w.rates, w.x0, w.times, seed=7)
    _vs_oracle(out, st, w, 7, "wave random 250x500")


def test_wave_kernel_exact_ssa(generic):
    w = gen.synthetic_workload(n_traj=100, t_end=0.5, n_samples=11)
    out, st = _vs_lanes(generic, w, 32, "wave exact SSA", method="ssa")
    _vs_oracle(out, st, w, 32, "wave exact SSA", method="ssa")


def test_wave_kernel_status_rules(generic):
    # max_steps mid-run, and an absorbing network
    w = gen.enzyme_workload(n_traj=200)
    out, st = _vs_lanes(generic, w, 33, "wave max_steps", max_steps=57)
    assert np.all(st[:, 3] & rn.ST_MAXSTEPS)
    d = gen.decay_network()
    wd = gen.Workload(name="decay", net=d, rates=np.full((1, 64), 2.0),
                      x0=np.array([5], np.int32), times=gen.sample_times(5.0, 6))
    out, st = _vs_lanes(generic, wd, 34, "wave absorbing decay")
    assert np.all(st[:, 3] & rn.ST_ABSORBED)
    _vs_oracle(out, st, wd, 34, "wave absorbing decay")


@pytest.mark.parametrize("name", ["synthetic", "stiff"])
def test_wave_kernel_fp32_equals_lanes(generic, name):
    w = (gen.synthetic_workload(n_traj=300, t_end=10.0, n_samples=21) if name == "synthetic"
         else gen.stiff_workload(n_traj=200))
    _vs_lanes(generic, w, 35, f"wave fp32 {w.name}", precision="fp32")


def test_wave_kernel_fp32_largest_network(generic):
    net = gen.random_network(3001, 250, 500)
    rng = np.random.default_rng(6)
    T = 64
    rates = gen.log_uniform(rng, 1e-4, 1.0, 500)[:, None] * gen.log_uniform(rng, 0.1, 10, (500, T))
    w = gen.Workload("random 250x500", net, np.ascontiguousarray(rates),
                     rng.integers(0, 1001, size=250).astype(np.int32), gen.sample_times(1.0, 6))
    _vs_lanes(generic, w, 36, "wave fp32 random 250x500", precision="fp32")


def test_wave_kernel_layout_range_and_statistics(generic, monkeypatch):
    # trajectory-major samples, a trajectory range with an offset, and the fused
    # sums, each against the same sweep in the default form
    import torch
    dev = torch.device("cuda:0")
    w = gen.synthetic_workload(n_traj=200, seed=3200, n_species=90, n_reactions=180, t_end=2.0,
                               n_samples=7)
    full, sfull = generic(w, 37, "wave")
    monkeypatch.setenv("RN_WSWEEP", "1")
    net = rn.Network(w.net)
    S, N = len(w.times), w.net.n_species
    a, b = 41, 173
    r = torch.from_numpy(np.ascontiguousarray(w.rates[:, a:b])).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o = torch.full((b - a, S, N), -1, dtype=torch.int32, device=dev)
    st = torch.zeros((b - a, 4), dtype=torch.int64, device=dev)
    sx = torch.full((S, N), 5, dtype=torch.int64, device=dev)
    sq = torch.full((S, N, 2), 5, dtype=torch.int64, device=dev)
    rn.sweep(net, r, x, tm, o, st, seed=37, traj_offset=a, out_layout="traj", sum_x=sx,
             sum_x2=sq)
    torch.cuda.synchronize()
    got = o.cpu().numpy().transpose(1, 2, 0)
    assert np.array_equal(got, full[:, :, a:b])
    assert np.array_equal(st.cpu().numpy().view(np.uint64), sfull[a:b])
    ref = full[:, :, a:b].astype(np.int64)
    assert np.array_equal(sx.cpu().numpy(), ref.sum(axis=2))
    q = sq.cpu().numpy().view(np.uint64)
    got2 = [int(u) + (int(v) << 64) for u, v in zip(q[..., 0].ravel(), q[..., 1].ravel())]
    assert got2 == [int(v) for v in (ref * ref).sum(axis=2).ravel()]
    _say("wave layout, range and statistics: identical")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wave_kernel_two_waves_per_simd(generic, precision):
    # more trajectories than the chip has SIMDs: the largest form (K = 8) runs
    # at two waves per SIMD, with registers spilled; still the same trajectories
    net = gen.random_network(3001, 250, 500)
    rng = np.random.default_rng(8)
    T = 1100
    rates = gen.log_uniform(rng, 1e-4, 1.0, 500)[:, None] * gen.log_uniform(rng, 0.1, 10, (500, T))
    w = gen.Workload("random 250x500", net, np.ascontiguousarray(rates),
                     rng.integers(0, 1001, size=250).astype(np.int32), gen.sample_times(0.5, 3))
    out, st = _vs_lanes(generic, w, 38, f"wave two waves per SIMD {precision}",
                        precision=precision)
    if precision == "fp64":
        for t in np.linspace(0, T - 1, 6).astype(int):
            ref, rst, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=38,
                                     traj_range=(int(t), int(t) + 1))
            assert np.array_equal(out[:, :, t], ref[:, :, 0]) and np.array_equal(st[t], rst[0])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wave_kernel_three_waves_per_simd(generic, precision):
    # the smallest form (K = 1) runs three waves per SIMD once the sweep
    # outnumbers the SIMDs; the 3-reaction enzyme network, 2,500 trajectories
    w = gen.enzyme_workload(n_traj=2500)
    out, st = _vs_lanes(generic, w, 39, f"wave three waves per SIMD {precision}",
                        precision=precision)
    if precision == "fp64":
        _vs_oracle(out, st, w, 39, "wave three waves per SIMD")
