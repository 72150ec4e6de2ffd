import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical test")


@pytest.fixture(autouse=True)
def _pin_lane_kernels(request, monkeypatch):
    # Small sweeps default to the one-wave-per-trajectory kernel; each GPU test
    # pins the kernel it exercises, so outside the modules that cover that
    # kernel and its choice, sweeps run one lane per trajectory (network-compiled
    # or generic).  A test that wants the default choice deletes the variable.
    if "wsweep" not in request.module.__name__ and "RN_WSWEEP" not in os.environ:
        monkeypatch.setenv("RN_WSWEEP", "0")
