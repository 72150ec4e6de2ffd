"""Fused ensemble statistics of rn_sweep (sum_x, sum_x2, hist): per (sample,
species), the exact integer sums of x and x^2 over the sweep's trajectories and
a histogram, accumulated by the sweep kernels as trajectories reach the sample
times, so that the sample array need not be written.

Sums and counts are integers, so they must equal exactly those of a sample
array: the oracle's where every trajectory is identical to the oracle's (the
FP64 parity cases), else the same sweep's own samples."""
import ctypes as C

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


def _host_stats(out, lo, width, bins):
    """Exact sums and histogram of an int32 [S][N][T] sample array."""
    x = out.astype(np.int64)
    sx = x.sum(axis=2)
    sq = (x * x).astype(object).sum(axis=2)  # exact beyond 2^63
    d = x - lo[None, :, None]
    b = np.where(d > 0, d // width[None, :, None], 0)
    b = np.minimum(b, bins - 1)
    S, N, _ = out.shape
    h = np.zeros((S, N, bins), np.int64)
    for s in range(S):
        for i in range(N):
            h[s, i] = np.bincount(b[s, i], minlength=bins)
    return sx, sq, h


def _fused(w, *, seed, with_out=True, precision="fp64", traj_offset=0, bins=16, lo=None,
           width=None, rates=None):
    """One sweep with fused statistics (and optionally the sample array)."""
    import torch

    dev = torch.device("cuda:0")
    net = rn.Network(w.net)
    rates = w.rates if rates is None else rates
    T, S, N = rates.shape[1], len(w.times), w.net.n_species
    if lo is None:
        lo = np.zeros(N, np.int32)
    if width is None:
        width = np.full(N, 64, np.int32)
    r = torch.from_numpy(np.ascontiguousarray(rates)).to(dev)
    x0 = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    out = torch.empty((S, N, T), dtype=torch.int32, device=dev) if with_out else None
    st = torch.empty((T, 4), dtype=torch.int64, device=dev)
    # stale contents: the call must clear them
    sx = torch.full((S, N), 12345, dtype=torch.int64, device=dev)
    sq = torch.full((S, N, 2), 777, dtype=torch.int64, device=dev)
    h = torch.full((S, N, bins), 99, dtype=torch.int32, device=dev)
    rn.sweep(net, r, x0, tm, out, st, seed=seed, eps=w.eps, n_c=w.n_c, precision=precision,
             traj_offset=traj_offset, sum_x=sx, sum_x2=sq, hist=h,
             hist_lo=torch.from_numpy(np.asarray(lo, np.int32)).to(dev),
             hist_width=torch.from_numpy(np.asarray(width, np.int32)).to(dev))
    torch.cuda.synchronize()
    q = sq.cpu().numpy().view(np.uint64)
    s2 = np.array([int(a) + (int(b) << 64) for a, b in zip(q[..., 0].ravel(), q[..., 1].ravel())],
                  dtype=object).reshape(S, N)
    return (out.cpu().numpy() if with_out else None, st.cpu().numpy().view(np.uint64),
            sx.cpu().numpy(), s2, h.cpu().numpy().astype(np.int64))


def _case(w, seed, bins=16, width=None):
    print(f"case stats {w.name}: T={w.n_traj} S={len(w.times)} N={w.net.n_species}", flush=True)
    width = np.full(w.net.n_species, 64, np.int32) if width is None else width
    lo = np.zeros(w.net.n_species, np.int32)
    out, st, sx, s2, h = _fused(w, seed=seed, bins=bins, width=width, lo=lo)
    ref, rst, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=seed, eps=w.eps, n_c=w.n_c,
                             threads=16)
    same = np.all(out == ref, axis=(0, 1)) & np.all(st == rst, axis=1)
    print(f"  identical trajectories {same.mean():.4f}", flush=True)
    base = ref if same.all() else out
    esx, esq, eh = _host_stats(base, lo, width, bins)
    assert np.array_equal(sx, esx), "sum of x differs"
    assert np.all(s2 == esq), "sum of x^2 differs"
    assert np.array_equal(h, eh), "histogram differs"
    assert np.all(h.sum(axis=2) == w.n_traj)
    # the same statistics without writing the samples
    _, st2, sx2, s22, h2 = _fused(w, seed=seed, with_out=False, bins=bins, width=width, lo=lo)
    assert np.array_equal(st2, st)
    assert np.array_equal(sx2, sx) and np.all(s22 == s2) and np.array_equal(h2, h)
    return out, st


def test_stats_enzyme():
    _case(gen.enzyme_workload(), 1, bins=32, width=np.array([4, 16, 4, 16], np.int32))


def test_stats_synthetic_ragged():
    _case(gen.synthetic_workload(n_traj=300, t_end=5.0, n_samples=21), 2)


def test_stats_stiff_subset():
    _case(gen.stiff_workload(n_traj=200), 4, bins=8)


def test_stats_generic_kernel_network(monkeypatch):
    # 70 species: the generic kernel records from its LDS counts
    monkeypatch.setenv("RN_WSWEEP", "0")
    w = gen.synthetic_workload(n_traj=257, n_species=70, n_reactions=140, t_end=2.0,
                               n_samples=9, seed=3)
    assert rn.sweep_kernel_kind(rn.Network(w.net), w.n_traj) == "generic"
    _case(w, 5)


def test_stats_large_counts_use_the_high_word():
    # counts near 2^31 make x^2 ~ 2^62: the 128-bit sum carries into its high word
    net = gen.source_network()
    T = 300
    rates = np.full((1, T), 1.0)
    times = np.array([0.0, 1.0, 2.0])
    w = gen.Workload(name="source_big", net=net, rates=rates,
                     x0=np.array([2_000_000_000], np.int32), times=times, seed=7)
    out, st, sx, s2, h = _fused(w, seed=7, bins=4, lo=np.array([1_999_999_990], np.int32),
                                width=np.array([4], np.int32))
    esx, esq, eh = _host_stats(out, np.array([1_999_999_990]), np.array([4]), 4)
    assert np.array_equal(sx, esx) and np.all(s2 == esq) and np.array_equal(h, eh)
    assert all(v >= (1 << 64) for v in s2.ravel())


def test_stats_fp32_equal_their_own_samples():
    w = gen.stiff_workload(n_traj=500)
    out, st, sx, s2, h = _fused(w, seed=9, precision="fp32")
    esx, esq, eh = _host_stats(out, np.zeros(30, np.int64), np.full(30, 64), 16)
    assert np.array_equal(sx, esx) and np.all(s2 == esq) and np.array_equal(h, eh)


def test_stats_of_ranges_add_up():
    w = gen.synthetic_workload(n_traj=400, n_species=12, n_reactions=24, t_end=3.0,
                               n_samples=7, seed=12)
    _, _, sx, s2, h = _fused(w, seed=3)
    a = 150
    _, _, sxa, s2a, ha = _fused(w, seed=3, rates=w.rates[:, :a])
    _, _, sxb, s2b, hb = _fused(w, seed=3, rates=w.rates[:, a:], traj_offset=a)
    assert np.array_equal(sxa + sxb, sx) and np.all(s2a + s2b == s2) and np.array_equal(ha + hb, h)


def test_stats_full_size_equal_moments_of_the_samples():
    # the benchmark sweep at full size (65,536 trajectories): the fused sums
    # equal rn_moments over the same launch's sample array
    import torch

    w = gen.synthetic_workload()
    print(f"case stats full size: T={w.n_traj}", flush=True)
    out, st, sx, s2, h = _fused(w, seed=w.seed)
    dev = torch.device("cuda:0")
    msx, msq = rn.moments(torch.from_numpy(out).to(dev), w.n_traj)
    torch.cuda.synchronize()
    m = msq.cpu().numpy().view(np.uint64)
    ms2 = np.array([int(a) + (int(b) << 64) for a, b in zip(m[..., 0].ravel(), m[..., 1].ravel())],
                   dtype=object).reshape(s2.shape)
    assert np.array_equal(sx, msx.cpu().numpy()) and np.all(s2 == ms2)
    assert np.all(h.sum(axis=2) == w.n_traj)


def test_stats_argument_errors():
    import torch

    w = gen.enzyme_workload(n_traj=8)
    dev = torch.device("cuda:0")
    net = rn.Network(w.net)
    r = torch.from_numpy(w.rates).to(dev)
    x0 = torch.from_numpy(w.x0).to(dev)
    tm = torch.from_numpy(w.times).to(dev)
    st = torch.empty((8, 4), dtype=torch.int64, device=dev)
    S, N = len(w.times), 4
    sx = torch.zeros((S, N), dtype=torch.int64, device=dev)
    a = rn.sweep_args(net, r, x0, tm, None, st, seed=1, sum_x=sx,
                      sum_x2=torch.zeros((S, N, 2), dtype=torch.int64, device=dev))
    a.sum_x2 = None  # sums must come together
    assert rn.lib().rn_sweep(net.handle, C.byref(a), None) == rn.RN_E_INVALID_ARG
    a.sum_x = None  # nothing to write at all
    assert rn.lib().rn_sweep(net.handle, C.byref(a), None) == rn.RN_E_INVALID_ARG
    a.hist = sx.data_ptr()  # a histogram without bins
    a.hist_bins = 0
    assert rn.lib().rn_sweep(net.handle, C.byref(a), None) == rn.RN_E_INVALID_ARG
