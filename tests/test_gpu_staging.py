"""Network tables reach the device with the first launch that uses them, on
that launch's stream: a handle used first on two streams at once, or first
inside a captured graph, must give the same results as a handle used on one
stream."""
import numpy as np
import pytest

from paper_1309_7695_amd import gen, rn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rn.lib()
    return torch, torch.device("cuda:0")


def _inputs(torch, dev, w):
    r = torch.from_numpy(w.rates).to(dev)
    x = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    S, N, T = len(w.times), w.net.n_species, w.n_traj
    return r, x, tm, S, N, T


def test_first_use_on_two_streams(torch_dev):
    torch, dev = torch_dev
    w = gen.synthetic_workload(n_traj=4096, seed=77, n_species=20, n_reactions=40, t_end=20.0,
                               n_samples=11)
    ref_out, ref_st = rn.run(w.net, w.rates, w.x0, w.times, seed=5)
    net = rn.Network(w.net)  # tables not on the device yet
    r, x, tm, S, N, T = _inputs(torch, dev, w)
    bufs = [(torch.empty((S, N, T), dtype=torch.int32, device=dev),
             torch.empty((T, 4), dtype=torch.int64, device=dev)) for _ in range(3)]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for (o, st), s in zip(bufs, (s1, s2, s1)):
        rn.sweep(net, r, x, tm, o, st, seed=5, stream=s)
    torch.cuda.synchronize()
    for k, (o, st) in enumerate(bufs):
        assert np.array_equal(o.cpu().numpy(), ref_out), k
        assert np.array_equal(st.cpu().numpy().view(np.uint64), ref_st), k
    print(f"  3 launches on two streams identical ({T} trajectories)", flush=True)


def test_first_use_inside_a_graph(torch_dev):
    torch, dev = torch_dev
    w = gen.synthetic_workload(n_traj=2048, seed=78, n_species=15, n_reactions=30, t_end=10.0,
                               n_samples=11)
    ref_out, ref_st = rn.run(w.net, w.rates, w.x0, w.times, seed=6)
    net = rn.Network(w.net)
    rn.sweep_kernel_kind(net, w.n_traj, "fp64")  # compile outside the capture
    r, x, tm, S, N, T = _inputs(torch, dev, w)
    o = torch.empty((S, N, T), dtype=torch.int32, device=dev)
    st = torch.empty((T, 4), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rn.sweep(net, r, x, tm, o, st, seed=6)
    for rep in range(3):
        o.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), ref_out), rep
        assert np.array_equal(st.cpu().numpy().view(np.uint64), ref_st), rep
    # the same handle outside the graph stages its tables itself
    o2 = torch.empty_like(o)
    st2 = torch.empty_like(st)
    rn.sweep(net, r, x, tm, o2, st2, seed=6)
    torch.cuda.synchronize()
    assert np.array_equal(o2.cpu().numpy(), ref_out)
    print("  graph replays and a later eager launch identical", flush=True)
