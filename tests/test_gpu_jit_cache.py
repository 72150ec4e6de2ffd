"""On-disk cache of network-compiled kernels (RN_JIT_CACHE): a second process
finds the code object its first run compiled and skips hipRTC; its results are
the same; a cache file whose stored compilation input differs is ignored."""
import glob
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, time
sys.path.insert(0, {root!r})
import numpy as np
from paper_1309_7695_amd import gen, rn
w = gen.synthetic_workload(n_traj=128, n_species=12, n_reactions=24, t_end=2.0, n_samples=5,
                           seed=4242)
net = rn.Network(w.net)
t0 = time.perf_counter()
kind = rn.sweep_kernel_kind(net, w.n_traj)
dt = time.perf_counter() - t0
out, st = rn.run(w.net, w.rates, w.x0, w.times, seed=3)
print("kind", kind, "setup", round(dt, 3), "digest", int(out.astype(np.int64).sum()),
      int(st.astype(np.int64).sum()), flush=True)
"""


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(cache):
    env = dict(os.environ, RN_JIT_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], capture_output=True,
                       text=True, timeout=300, env=env)
    print(r.stdout, r.stderr[-800:], flush=True)
    assert r.returncode == 0
    line = [l for l in r.stdout.splitlines() if l.startswith("kind")][-1].split()
    return line[1], float(line[3]), line[5:]


def test_second_process_loads_the_cached_kernel(tmp_path):
    kind1, t1, d1 = _run(tmp_path)
    files = glob.glob(str(tmp_path / "rn_*.co"))
    assert kind1 == "network" and len(files) == 1
    kind2, t2, d2 = _run(tmp_path)
    print(f"compile {t1:.2f} s, cached {t2:.2f} s", flush=True)
    assert kind2 == "network" and d2 == d1
    assert t2 < t1 / 2
    # a file whose stored input differs is not used: the kernel is compiled again
    data = open(files[0], "rb").read()
    bad = bytearray(data)
    bad[20] ^= 0xFF
    open(files[0], "wb").write(bytes(bad))
    kind3, t3, d3 = _run(tmp_path)
    assert kind3 == "network" and d3 == d1
    # rewritten by the fresh compilation: the stored input is whole again
    assert open(files[0], "rb").read()[:4096] == data[:4096]
