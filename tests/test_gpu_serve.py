"""The sweep-job server (rn_server): jobs of different networks and sizes,
admitted in a tight HBM budget so that some wait for others, must each give
exactly the results the same job gives alone through rn_sweep, in FP64 and in
FP32 (the server may pick the generic or the network-compiled kernel, which
are identical)."""
import sys
import time

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


def _job_bytes(w):
    S, N, T, M = len(w.times), w.net.n_species, w.n_traj, w.net.n_reactions
    r = lambda b: (b + 255) // 256 * 256
    return r(M * T * 8) + r(N * 4) + r(S * 8) + r(S * N * T * 4) + r(T * 32)


@pytest.mark.parametrize("choice", ["lanes", "default"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_server_mix_equals_alone(precision, choice, monkeypatch):
    # "default": the library's kernel choice, which runs these small jobs one
    # wave per trajectory (the reference sweeps below then run the same way)
    if choice == "default":
        monkeypatch.delenv("RN_WSWEEP", raising=False)
    arrivals, ws = gen.serve_jobs(n_jobs=8, seed=5100, t_scale=0.02, t_end_scale=0.02,
                                  n_samples=11)
    budget = int(1.5 * max(_job_bytes(w) for w in ws))  # forces queueing
    nets = [rn.Network(w.net) for w in ws]
    _say(f"server {precision}: T={[w.n_traj for w in ws]} M={[w.net.n_reactions for w in ws]} "
         f"budget {budget} B")
    srv = rn.Server(budget, max_running=3)
    ids = [srv.submit(nets[k], w.rates, w.x0, w.times, seed=40 + k, precision=precision)
           for k, w in enumerate(ws)]
    saw_queue = srv.status()["queued"] > 0
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        for jid in srv.poll():
            got[jid] = srv.fetch(jid)
        saw_queue = saw_queue or srv.status()["queued"] > 0
        assert time.time() - t0 < 240, "server made no progress"
        time.sleep(0.001)
    assert saw_queue
    assert srv.status() == {"queued": 0, "running": 0, "bytes_in_use": 0}
    srv.close()
    for k, w in enumerate(ws):
        out, st = rn.run(nets[k], w.rates, w.x0, w.times, seed=40 + k, precision=precision)
        assert np.array_equal(got[ids[k]][0], out), k
        assert np.array_equal(got[ids[k]][1], st), k
    _say(f"  {len(ws)} jobs identical in the mix and alone")


def test_server_rejects_job_over_budget():
    w = gen.synthetic_workload(n_traj=1000, n_species=10, n_reactions=20, t_end=1.0,
                               n_samples=11)
    srv = rn.Server(_job_bytes(w) // 2, max_running=1)
    with pytest.raises(rn.RNError) as e:
        srv.submit(rn.Network(w.net), w.rates, w.x0, w.times, seed=1)
    assert e.value.code == rn.RN_E_NOMEM
    srv.close()


def test_server_pinned_results_free_the_device_block():
    """With staging room for every whole job, each job's results go to pinned
    host memory on its own stream: the device budget is free again as soon as
    the jobs complete (before any fetch), and the fetched results equal the
    same jobs run alone."""
    arrivals, ws = gen.serve_jobs(n_jobs=6, seed=5200, t_scale=0.02, t_end_scale=0.02,
                                  n_samples=11)
    budget = 8 * sum(_job_bytes(w) for w in ws)  # staging area: 2x all jobs
    nets = [rn.Network(w.net) for w in ws]
    srv = rn.Server(budget, max_running=4)
    ids = [srv.submit(nets[k], w.rates, w.x0, w.times, seed=60 + k) for k, w in enumerate(ws)]
    done = set()
    t0 = time.time()
    while len(done) < len(ids):
        done.update(srv.poll())
        assert time.time() - t0 < 240, "server made no progress"
        time.sleep(0.001)
    assert srv.status() == {"queued": 0, "running": 0, "bytes_in_use": 0}
    got = {jid: srv.fetch(jid) for jid in ids}
    srv.close()
    for k, w in enumerate(ws):
        out, st = rn.run(nets[k], w.rates, w.x0, w.times, seed=60 + k)
        assert np.array_equal(got[ids[k]][0], out), k
        assert np.array_equal(got[ids[k]][1], st), k
    _say(f"  {len(ws)} jobs with pinned results identical to alone")
