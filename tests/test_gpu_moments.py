"""Ensemble moments (rn_moments) against their definition: exact integer sums
over trajectories of every (sample, species) row."""
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
    return torch.device("cuda:0")


def _exact(out):
    o = out.astype(np.int64)
    s1 = o.sum(axis=2)
    s2 = np.array([[sum(int(v) * int(v) for v in o[s, i]) for i in range(o.shape[1])]
                   for s in range(o.shape[0])], dtype=object)
    return s1, s2


def _split(s2):
    w = s2.cpu().numpy().view(np.uint64)
    return np.array([[int(w[s, i, 0]) + (int(w[s, i, 1]) << 64) for i in range(w.shape[1])]
                     for s in range(w.shape[0])], dtype=object)


@pytest.mark.parametrize("T", [1, 63, 300, 301, 1029])
def test_moments_of_arbitrary_counts_are_exact(T):
    import torch
    rng = np.random.default_rng(T)
    S, N = 3, 5
    vals = rng.integers(-2**31, 2**31, size=(S, N, T), dtype=np.int64).astype(np.int32)
    vals[0, 0, :] = 2**31 - 1          # worst case for the 128-bit sum of squares
    vals[0, 1, :] = -2**31
    o = torch.from_numpy(vals).cuda()
    sx, sq = rn.moments(o)
    torch.cuda.synchronize()
    s1, s2 = _exact(vals)
    assert np.array_equal(sx.cpu().numpy(), s1)
    assert (_split(sq) == s2).all()


def test_moments_of_padded_rows_use_only_n_traj():
    import torch
    vals = np.arange(2 * 3 * 40, dtype=np.int32).reshape(2, 3, 40)
    o = torch.from_numpy(vals).cuda()
    sx, sq = rn.moments(o, n_traj=37)
    torch.cuda.synchronize()
    s1, s2 = _exact(vals[:, :, :37])
    assert np.array_equal(sx.cpu().numpy(), s1)
    assert (_split(sq) == s2).all()


def test_moments_of_a_sweep_match_the_oracle_ensemble():
    import torch
    w = gen.enzyme_workload()
    net = rn.Network(w.net)
    dev = torch.device("cuda:0")
    o = torch.empty((len(w.times), 4, w.n_traj), dtype=torch.int32, device=dev)
    s = torch.empty((w.n_traj, 4), dtype=torch.int64, device=dev)
    rn.sweep(net, torch.from_numpy(w.rates).to(dev), torch.from_numpy(w.x0).to(dev),
             torch.from_numpy(w.times).to(dev), o, s, seed=1)
    sx, sq = rn.moments(o)
    torch.cuda.synchronize()
    ref, _, _ = oracle.run(w.net, w.rates, w.x0, w.times, seed=1, threads=8)
    s1, s2 = _exact(ref)
    assert np.array_equal(sx.cpu().numpy(), s1)
    assert (_split(sq) == s2).all()
    mean, var, _ = rn.moment_stats(sx.cpu().numpy(), sq.cpu().numpy(), w.n_traj)
    assert np.allclose(mean, ref.mean(axis=2), rtol=0, atol=1e-12)
    assert np.allclose(var, ref.astype(np.float64).var(axis=2, ddof=1), rtol=1e-12, atol=1e-9)


def test_moments_argument_errors():
    import ctypes as C
    L = rn.lib()
    assert L.rn_moments(None, 1, 1, 1, 1, None, None, None) == rn.RN_E_INVALID_ARG
