"""Batched sweeps (rn_batch): jobs of uneven network and trajectory count,
recorded once into a HIP graph and replayed.  Each job's results must equal,
bit for bit, those of rn_sweep with the same arguments (rn_sweep itself is
checked against the oracle in test_gpu_parity.py).  Graph replays are checked
one by one, with eager work and synchronizations between them."""
import sys

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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _jobs():
    import torch
    dev = torch.device("cuda:0")
    # uneven sizes: four networks of 10-300 reactions (one too large for the
    # network-compiled kernel is appended), 40-700 trajectories each
    ws = gen.batch_workloads(n_networks=4, seed=3100, m_range=(10, 300), t_range=(40, 700),
                             t_end=4.0, n_samples=9)
    ws.append(gen.synthetic_workload(n_traj=150, seed=3200, n_species=90, n_reactions=180,
                                     t_end=1.0, n_samples=5))
    jobs = []
    for k, w in enumerate(ws):
        net = rn.Network(w.net)
        S, N, T = len(w.times), w.net.n_species, w.n_traj
        jobs.append(dict(
            w=w, net=net, seed=77 + k,
            rates=torch.from_numpy(w.rates).to(dev), x0=torch.from_numpy(w.x0).to(dev),
            times=torch.from_numpy(w.times).to(dev),
            out=torch.full((S, N, T), -1, dtype=torch.int32, device=dev),
            stats=torch.zeros((T, 4), dtype=torch.int64, device=dev)))
    kinds = rn.precompile([j["net"] for j in jobs], [j["w"].n_traj for j in jobs])
    _say(f"batch jobs: M={[j['w'].net.n_reactions for j in jobs]} "
         f"T={[j['w'].n_traj for j in jobs]} kernels={kinds}")
    assert "network" in kinds and "generic" in kinds
    return jobs


def test_batch_equals_individual_sweeps_over_replays():
    import torch
    jobs = _jobs()
    ref = []
    for j in jobs:
        rn.sweep(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"])
        torch.cuda.synchronize()
        ref.append((j["out"].cpu().numpy().copy(), j["stats"].cpu().numpy().copy()))
    b = rn.Batch()
    for j in jobs:
        b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"])
    assert len(b) == len(jobs)
    for rep in range(3):
        for j in jobs:  # clear the outputs eagerly, outside the graph
            j["out"].fill_(-1)
            j["stats"].zero_()
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for k, j in enumerate(jobs):
            assert np.array_equal(j["out"].cpu().numpy(), ref[k][0]), (rep, k)
            assert np.array_equal(j["stats"].cpu().numpy(), ref[k][1]), (rep, k)
        _say(f"replay {rep}: {len(jobs)} jobs identical to rn_sweep")
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda:0")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum()).item()
    b.close()


def test_batch_rejects_jobs_after_launch():
    import torch
    jobs = _jobs()[:1]
    j = jobs[0]
    b = rn.Batch()
    b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=1)
    b.launch()
    torch.cuda.synchronize()
    with pytest.raises(rn.RNError):
        b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=2)
    b.close()
