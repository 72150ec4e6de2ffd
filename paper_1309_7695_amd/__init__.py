"""MI355X-native (gfx950) tau-leaping parameter sweeps of mass-action reaction networks.

The compute path is the HIP library ``librn.so`` (C ABI in ``include/rn.h``),
reached through the ctypes binding in :mod:`paper_1309_7695_amd.rn`.
Seeded synthetic inputs live in :mod:`paper_1309_7695_amd.gen`.
"""
from . import gen, rn  # noqa: F401

__all__ = ["gen", "rn"]
