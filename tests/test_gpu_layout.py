"""The trajectory-major output layout (RN_OUT_TRAJ_MAJOR): out[t][s][i] holds
exactly what the default layout holds at out[s][i][t], for every kernel that
writes samples (network-compiled, generic, exact-SSA with a dependency graph),
in both precisions, and for trajectory ranges written into a wider array."""
import os

import numpy as np
import pytest

from paper_1309_7695_amd import gen, rn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rn.lib()


def _both(w, seed, **kw):
    import torch
    dev = torch.device("cuda:0")
    net = rn.Network(w.net)
    T, S, N = w.n_traj, len(w.times), w.net.n_species
    r = torch.from_numpy(w.rates).to(dev)
    x0 = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    o1 = torch.full((S, N, T), -1, dtype=torch.int32, device=dev)
    s1 = torch.zeros((T, 4), dtype=torch.int64, device=dev)
    rn.sweep(net, r, x0, tm, o1, s1, seed=seed, **kw)
    o2 = torch.full((T, S, N), -1, dtype=torch.int32, device=dev)
    s2 = torch.zeros((T, 4), dtype=torch.int64, device=dev)
    rn.sweep(net, r, x0, tm, o2, s2, seed=seed, out_layout="traj", **kw)
    torch.cuda.synchronize()
    a, b = o1.cpu().numpy(), o2.cpu().numpy()
    assert np.array_equal(s1.cpu().numpy(), s2.cpu().numpy())
    assert np.array_equal(a, b.transpose(1, 2, 0)), "layouts hold different samples"
    return a


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_traj_major_network_kernel(precision):
    w = gen.synthetic_workload(n_traj=300, t_end=3.0, n_samples=13)
    print(f"case layout {w.name} {precision}", flush=True)
    _both(w, 5, precision=precision)


def test_traj_major_full_workgroups():
    # 256-lane workgroups (four waves)
    w = gen.synthetic_workload(n_traj=65536, t_end=0.2, n_samples=5)
    print(f"case layout full workgroups {w.name}", flush=True)
    _both(w, 6)


def test_traj_major_generic_kernel(monkeypatch):
    monkeypatch.setenv("RN_WSWEEP", "0")
    w = gen.synthetic_workload(n_traj=257, n_species=70, n_reactions=140, t_end=1.0,
                               n_samples=6, seed=3)
    assert rn.sweep_kernel_kind(rn.Network(w.net), w.n_traj) == "generic"
    _both(w, 7)


def test_traj_major_ssa_dependency_kernel():
    old = os.environ.get("RN_SSA_KERNEL")
    os.environ["RN_SSA_KERNEL"] = "dep"
    try:
        _both(gen.enzyme_workload(n_traj=200), 8, method=rn.METHOD_SSA)
    finally:
        if old is None:
            del os.environ["RN_SSA_KERNEL"]
        else:
            os.environ["RN_SSA_KERNEL"] = old


def test_traj_major_range_into_wider_rows():
    # trajectories [a, b) of a sweep, written with a row stride wider than S*N
    import torch
    dev = torch.device("cuda:0")
    w = gen.synthetic_workload(n_traj=200, n_species=10, n_reactions=20, t_end=2.0, n_samples=5)
    full = _both(w, 9)
    net = rn.Network(w.net)
    a, b = 37, 151
    S, N = len(w.times), 10
    wide = torch.full((b - a, S * N + 7), -1, dtype=torch.int32, device=dev)
    view = torch.as_strided(wide, (b - a, S, N), (S * N + 7, N, 1))
    st = torch.zeros((b - a, 4), dtype=torch.int64, device=dev)
    rn.sweep(net, torch.from_numpy(np.ascontiguousarray(w.rates[:, a:b])).to(dev),
             torch.from_numpy(w.x0).to(dev), torch.from_numpy(w.times).to(dev), view, st,
             seed=9, traj_offset=a, out_layout="traj")
    torch.cuda.synchronize()
    got = view.cpu().numpy()
    assert np.array_equal(got.transpose(1, 2, 0), full[:, :, a:b])
    assert np.all(wide.cpu().numpy()[:, S * N:] == -1)  # the padding is untouched
