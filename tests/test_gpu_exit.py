"""A process that exits while network-kernel compilations are still queued or
running in the background must exit cleanly.

rn_server_submit starts compiling the job's network kernel on a worker thread.
A compilation still inside hipRTC while the process tears down its libraries
used to crash the exit; the binding now drains the compile pool at interpreter
exit, and the pool's own destructor drains it for C callers.  Each case runs in
a fresh subprocess and must return 0."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
from paper_1309_7695_amd import gen, rn
jobs = []
srv = rn.Server(1 << 28, max_running=2)
for k in range(6):
    w = gen.synthetic_workload(n_traj=64, n_species=20 + k, n_reactions=40 + 2 * k, t_end=0.01,
                               n_samples=2, seed=9100 + k)
    net = rn.Network(w.net)
    jobs.append((net, srv.submit(net, w.rates, w.x0, w.times, seed=k)))
print("submitted", len(jobs), flush=True)
{tail}
"""


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# exit at once; free the server first; exit without the binding's drain (the
# pool's destructor drains it, as for a C caller that never calls it)
@pytest.mark.parametrize("tail", ["pass", "srv.close()",
                                  "import atexit; atexit.unregister(rn.lib().rn_compile_drain)"])
def test_exit_with_background_compiles_queued(tail):
    code = SCRIPT.format(root=ROOT, tail=tail)
    print(f"case exit with queued compiles, tail {tail!r}", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=180)
    print(r.stdout[-500:], r.stderr[-1500:], flush=True)
    assert "submitted 6" in r.stdout
    assert r.returncode == 0, r.returncode
