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
    assert "network" in kinds and set(kinds) - {"network"}
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


def _batch_matches(jobs, ref, b, label, extra=None):
    import torch
    for rep in range(3):
        for j in jobs:  # clear the outputs eagerly, outside the graph
            j["out"].fill_(-1)
            j["stats"].zero_()
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for k, j in enumerate(jobs):
            assert np.array_equal(j["out"].cpu().numpy(), ref[k][0]), (label, rep, k)
            assert np.array_equal(j["stats"].cpu().numpy(), ref[k][1]), (label, rep, k)
        if extra is not None:
            extra(rep)
        _say(f"{label} replay {rep}: {len(jobs)} jobs identical to rn_sweep")
        x = torch.randn(1 << 20, device="cuda:0")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum()).item()


def _reference(jobs, **kw):
    import torch
    ref = []
    for j in jobs:
        rn.sweep(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"],
                 **kw)
        torch.cuda.synchronize()
        ref.append((j["out"].cpu().numpy().copy(), j["stats"].cpu().numpy().copy()))
    return ref


def test_persistent_batch_equals_individual_sweeps_over_replays():
    # one persistent kernel per launch shape over a (job, block) queue; every
    # job bit for bit the trajectories rn_sweep gives (network-compiled or not)
    jobs = _jobs()
    ref = _reference(jobs)
    b = rn.Batch(persistent=True)
    for j in jobs:
        b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"])
    _batch_matches(jobs, ref, b, "persistent")
    b.close()


def test_persistent_batch_fp32_and_fused_statistics():
    import torch
    jobs = _jobs()[:3]
    ref = _reference(jobs, precision="fp32")
    dev = torch.device("cuda:0")
    sums = []
    b = rn.Batch(persistent=True)
    for j in jobs:
        S, N = len(j["w"].times), j["w"].net.n_species
        sx = torch.zeros((S, N), dtype=torch.int64, device=dev)
        sq = torch.zeros((S, N, 2), dtype=torch.int64, device=dev)
        sums.append((sx, sq))
        b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"],
              precision="fp32", sum_x=sx, sum_x2=sq)

    def check_sums(rep):
        for k, j in enumerate(jobs):
            o = ref[k][0].astype(np.int64)
            assert np.array_equal(sums[k][0].cpu().numpy(), o.sum(axis=2)), (rep, k)
            q = sums[k][1].cpu().numpy().view(np.uint64)
            got = [int(a) + (int(c) << 64) for a, c in zip(q[..., 0].ravel(), q[..., 1].ravel())]
            want = [int(v) for v in (o * o).sum(axis=2).ravel()]
            assert got == want, (rep, k)

    _batch_matches(jobs, ref, b, "persistent fp32 + statistics", check_sums)
    b.close()


def test_tuned_persistent_batch_and_cache_file(tmp_path, monkeypatch):
    # the autotuner's choices change launch shapes only: results stay those of
    # rn_sweep; the choices are written to RN_TUNE_CACHE
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("RN_TUNE_CACHE", str(cache))
    jobs = _jobs()
    ref = _reference(jobs)
    b = rn.Batch(persistent=True)
    for j in jobs:
        b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"])
    b.tune()
    lines = cache.read_text().split("\n")
    rows = [l.split() for l in lines if l.strip()]
    _say(f"tuned buckets: {rows}")
    assert rows and all(len(r) == 7 and r[4] in ("64", "256") for r in rows)
    _batch_matches(jobs, ref, b, "tuned persistent")
    b.close()


def test_persistent_switch_rejected_after_launch():
    import torch
    j = _jobs()[0]
    b = rn.Batch()
    b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=1)
    b.launch()
    torch.cuda.synchronize()
    assert rn.lib().rn_batch_persistent(b.handle, 1) == rn.RN_E_INVALID_ARG
    assert rn.lib().rn_batch_tune(b.handle, None) == rn.RN_E_INVALID_ARG
    b.close()


RATES_FROM_MEMORY = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import torch
from paper_1309_7695_amd import gen, rn
dev = torch.device("cuda:0")
ws = [gen.synthetic_workload(n_traj=300, t_end=2.0, n_samples=7, seed=3301),
      gen.synthetic_workload(n_traj=130, n_species=18, n_reactions=37, t_end=3.0, n_samples=6,
                             seed=3302)]
for prec in ("fp64", "fp32"):
    jobs, ref = [], []
    for k, w in enumerate(ws):
        net = rn.Network(w.net)
        S, N, T = len(w.times), w.net.n_species, w.n_traj
        j = dict(net=net, rates=torch.from_numpy(w.rates).to(dev),
                 x0=torch.from_numpy(w.x0).to(dev),
                 times=torch.from_numpy(w.times).to(dev),
                 out=torch.full((S, N, T), -1, dtype=torch.int32, device=dev),
                 stats=torch.zeros((T, 4), dtype=torch.int64, device=dev), seed=91 + k)
        rn.sweep(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"],
                 precision=prec)
        torch.cuda.synchronize()
        ref.append((j["out"].cpu().numpy().copy(), j["stats"].cpu().numpy().copy()))
        j["out"].fill_(-1)
        j["stats"].zero_()
        jobs.append(j)
    b = rn.Batch(persistent=True)
    for j in jobs:
        b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"], seed=j["seed"],
              precision=prec)
    b.launch()
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        assert np.array_equal(j["out"].cpu().numpy(), ref[k][0]), (prec, k)
        assert np.array_equal(j["stats"].cpu().numpy(), ref[k][1]), (prec, k)
    b.close()
    print("identical", prec, flush=True)
"""


def _bucket(w, precision):
    # (precision, species/8, reactions/16, nonzero net changes/32): the tuner's key
    nnz = 0
    for re, pr in zip(w.net.reactants, w.net.products):
        d = {}
        for s, c in re:
            d[s] = d.get(s, 0) - c
        for s, c in pr:
            d[s] = d.get(s, 0) + c
        nnz += sum(1 for v in d.values() if v != 0)
    return (precision, (w.net.n_species + 7) // 8, (w.net.n_reactions + 15) // 16,
            (nnz + 31) // 32)


def test_persistent_rates_from_memory_on_padded_networks(tmp_path):
    # a tuned shape may read the rate constants from memory (no rate registers)
    # for a network whose reaction count is padded to whole rate vectors: the
    # padding reactions have no rows in the rates array and must count as rate
    # 0, exactly as in the register form
    import os
    import subprocess
    ws = [gen.synthetic_workload(n_traj=300, t_end=2.0, n_samples=7, seed=3301),
          gen.synthetic_workload(n_traj=130, n_species=18, n_reactions=37, t_end=3.0,
                                 n_samples=6, seed=3302)]
    assert all(w.net.n_reactions % 16 for w in ws)
    cache = tmp_path / "tune.txt"
    rows = [_bucket(w, p) for w in ws for p in (0, 1)]
    cache.write_text("".join(f"{a} {b} {c} {d} 64 0 0.500\n" for a, b, c, d in rows))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, RN_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", RATES_FROM_MEMORY.format(root=root)],
                       capture_output=True, text=True, timeout=300, env=env)
    _say(r.stdout + r.stderr[-1500:])
    assert r.returncode == 0
    assert "identical fp64" in r.stdout and "identical fp32" in r.stdout


def test_default_kernel_choice_in_both_batch_forms(monkeypatch):
    # with the default choice, small jobs run one wave per trajectory: the graph
    # and the persistent form (which puts those jobs on their own branches)
    # still give every job exactly rn_sweep's results
    jobs = _jobs()  # (built with the lane kernels pinned)
    monkeypatch.delenv("RN_WSWEEP", raising=False)
    kinds = [rn.sweep_kernel_kind(j["net"], j["w"].n_traj) for j in jobs]
    _say(f"default kernel choice: {kinds}")
    assert "wave" in kinds
    ref = _reference(jobs)
    for persistent in (False, True):
        b = rn.Batch(persistent=persistent)
        for j in jobs:
            b.add(j["net"], j["rates"], j["x0"], j["times"], j["out"], j["stats"],
                  seed=j["seed"])
        _batch_matches(jobs, ref, b, f"default choice, persistent={persistent}")
        b.close()
