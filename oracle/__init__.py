"""Plain FP64 CPU oracle for tau-leaping parameter sweeps (ctypes binding).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, by the package smoke
check and by the benchmark's CPU-baseline leg; the product path never imports
it.  It shares no code with the HIP path: its own C source computes the
network tables, the Philox stream, the samplers and the method's steps.

The method is Cao-Gillespie-Petzold tau-leaping with critical reactions and an
exact-SSA fallback (Cao, Gillespie, Petzold, J. Chem. Phys. 124, 044109, 2006)
applied to the stochastic model of the paper's Methods section.
"""
from __future__ import annotations

import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

ST_ABSORBED, ST_MAXSTEPS, ST_OVERFLOW = 1, 2, 4


class _NetDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("react_ptr", C.c_void_p), ("react_species", C.c_void_p), ("react_coeff", C.c_void_p),
                ("prod_ptr", C.c_void_p), ("prod_species", C.c_void_p), ("prod_coeff", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("eps", C.c_double), ("n_c", C.c_int32),
                ("ssa_factor", C.c_double), ("ssa_burst", C.c_int32),
                ("max_steps", C.c_uint64), ("method", C.c_int32), ("cle_threshold", C.c_double)]


class _OdeParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_uint64),
                ("method", C.c_int32)]


class _HybridParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("rtol", C.c_double), ("atol", C.c_double),
                ("max_steps", C.c_uint64)]


OPS_FIELDS = ["leaps", "ssa_events", "rejections", "prop_evals", "crit_tests", "tau_terms",
              "tau_species", "philox_blocks", "inv_draws", "inv_iters", "ptrs_draws",
              "ptrs_iters", "ptrs_log_tests", "exp_draws", "select_terms", "update_terms"]


class _Ops(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in OPS_FIELDS]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_philox4x32_10.restype = None
        L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u53.restype = C.c_double
        L.orc_poisson.argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32,
                                  C.c_void_p]
        L.orc_poisson.restype = C.c_int64
        L.orc_poisson_many.argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_int32, C.c_int64,
                                       C.c_void_p]
        L.orc_poisson_many.restype = None
        L.orc_cle_many.argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_int32, C.c_int64,
                                   C.c_void_p]
        L.orc_cle_many.restype = None
        L.orc_pick_index.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p]
        L.orc_pick_index.restype = C.c_int
        L.orc_critical_fires.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_critical_fires.restype = C.c_int
        L.orc_run.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_run.restype = C.c_int
        L.orc_ode_run.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                  C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int64,
                                  C.c_void_p, C.c_void_p]
        L.orc_ode_run.restype = C.c_int
        L.orc_hybrid_run.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_int64, C.c_void_p, C.c_int32, C.c_int64, C.c_int64,
                                     C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_hybrid_run.restype = C.c_int
        _lib = L
    return _lib


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def u53(hi, lo):
    return lib().orc_u53(int(hi), int(lo))


def poisson(lam, seed, traj, n, j):
    return int(lib().orc_poisson(float(lam), int(seed), int(traj), int(n), int(j), None))


def poisson_many(lam, seed, n, j=0, n0=0):
    out = np.zeros(int(n), dtype=np.int64)
    lib().orc_poisson_many(float(lam), int(seed), int(n0), int(j), int(n), out.ctypes.data)
    return out


def pick_index(a, r, allowed=None):
    """The direct method's selection over the propensities ``a`` for ``r``."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    al = None if allowed is None else np.ascontiguousarray(allowed, dtype=np.int32)
    return int(lib().orc_pick_index(a.ctypes.data, len(a), float(r),
                                    None if al is None else al.ctypes.data))


def critical_fires(tau_c, tau_p, delta):
    """1 when the critical race is won (see ``orc_critical_fires``)."""
    return int(lib().orc_critical_fires(float(tau_c), float(tau_p), float(delta)))


def _desc(net):
    arrs = {k: np.ascontiguousarray(v, dtype=np.int32) for k, v in net.csr().items()}
    d = _NetDesc(net.n_species, net.n_reactions,
                 arrs["react_ptr"].ctypes.data, arrs["react_species"].ctypes.data,
                 arrs["react_coeff"].ctypes.data, arrs["prod_ptr"].ctypes.data,
                 arrs["prod_species"].ctypes.data, arrs["prod_coeff"].ctypes.data)
    return d, arrs


def cle_many(lam, seed, n, j=0, n0=0):
    out = np.zeros(int(n), dtype=np.int64)
    lib().orc_cle_many(float(lam), int(seed), int(n0), int(j), int(n), out.ctypes.data)
    return out


def run(net, rates, x0, times, *, seed, eps=0.03, n_c=10, ssa_factor=10.0, ssa_burst=100,
        max_steps=10**8, method="tauleap", traj_range=None, threads=1, counters=False,
        cle_threshold=0.0):
    """Simulate trajectories ``traj_range = (a, b)`` (default: all columns of ``rates``).

    Returns ``(out, stats, ops)``: ``out`` int32 ``[S][N][b-a]``, ``stats`` uint64
    ``[b-a][4]`` (leaps, ssa events, rejections, status bits) and ``ops`` a dict
    of operation counts (or None).
    """
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    M, T = rates.shape
    if M != net.n_reactions:
        raise ValueError("rates must have one row per reaction")
    a, b = traj_range if traj_range is not None else (0, T)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    if x0.ndim == 2 and x0.shape[1] != T:
        raise ValueError("per-trajectory x0 must have one column per trajectory")
    times = np.ascontiguousarray(times, dtype=np.float64)
    S, N = len(times), net.n_species
    n = b - a
    out = np.zeros((S, N, n), dtype=np.int32)
    stats = np.zeros((n, 4), dtype=np.uint64)
    desc, keep = _desc(net)
    par = _Params(int(seed), float(eps), int(n_c), float(ssa_factor), int(ssa_burst),
                  int(max_steps), 1 if method == "ssa" else 0, float(cle_threshold))
    L = lib()
    chunks = []
    nth = max(1, min(int(threads), n)) if n > 0 else 1
    bounds = np.linspace(0, n, nth + 1).astype(np.int64)
    ops_list = [_Ops() for _ in range(nth)]

    def work(ci):
        lo, hi = int(bounds[ci]), int(bounds[ci + 1])
        if hi <= lo:
            return 0
        rp = rates.ctypes.data + 8 * (a + lo)
        if x0.ndim == 2:
            xp, xld = x0.ctypes.data + 4 * (a + lo), T
        else:
            xp, xld = x0.ctypes.data, 0
        # out[(s*N+i)*n + t] with t offset by lo
        op = out.ctypes.data + 4 * lo
        sp = stats.ctypes.data + 8 * 4 * lo
        return L.orc_run(C.byref(desc), rp, T, xp, xld, times.ctypes.data, S, a + lo, hi - lo,
                         op, n, sp, C.byref(par), C.byref(ops_list[ci]) if counters else None)

    if nth == 1:
        rcs = [work(0)]
    else:
        with ThreadPoolExecutor(nth) as ex:
            rcs = list(ex.map(work, range(nth)))
    for rc in rcs:
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}")
    del chunks, keep
    ops = None
    if counters:
        ops = {f: sum(getattr(o, f) for o in ops_list) for f in OPS_FIELDS}
    return out, stats, ops


ODE_METHODS = {"dopri5": 0, "ros4": 1}


def ode_run(net, rates, x0, times, *, rtol=1e-6, atol=1e-6, max_steps=10**7, traj_range=None,
            threads=1, method="dopri5"):
    """Reaction-rate equations for trajectories ``traj_range``, by the
    Dormand-Prince 5(4) pair (``method="dopri5"``) or the Rosenbrock 4(3)
    method for stiff networks (``method="ros4"``).

    Returns ``(out [S][N][T] float64, stats [T][4] uint64)`` with stats = (accepted
    steps, rejected steps, 0, status)."""
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    M, T = rates.shape
    a, b = traj_range if traj_range is not None else (0, T)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    times = np.ascontiguousarray(times, dtype=np.float64)
    S, N = len(times), net.n_species
    n = b - a
    out = np.zeros((S, N, n), dtype=np.float64)
    stats = np.zeros((n, 4), dtype=np.uint64)
    desc, keep = _desc(net)
    par = _OdeParams(float(rtol), float(atol), int(max_steps), ODE_METHODS[method])
    L = lib()
    nth = max(1, min(int(threads), n)) if n > 0 else 1
    bounds = np.linspace(0, n, nth + 1).astype(np.int64)

    def work(ci):
        lo, hi = int(bounds[ci]), int(bounds[ci + 1])
        if hi <= lo:
            return 0
        rp = rates.ctypes.data + 8 * (a + lo)
        if x0.ndim == 2:
            xp, xld = x0.ctypes.data + 4 * (a + lo), T
        else:
            xp, xld = x0.ctypes.data, 0
        return L.orc_ode_run(C.byref(desc), rp, T, xp, xld, times.ctypes.data, S, hi - lo,
                             out.ctypes.data + 8 * lo, n, stats.ctypes.data + 32 * lo, C.byref(par))

    if nth == 1:
        rcs = [work(0)]
    else:
        with ThreadPoolExecutor(nth) as ex:
            rcs = list(ex.map(work, range(nth)))
    for rc in rcs:
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}")
    del keep
    return out, stats


def hybrid_run(net, continuous, rates, x0, times, *, seed, rtol=1e-6, atol=1e-6,
               max_steps=10**7, traj_range=None, threads=1):
    """Hybrid stochastic/deterministic sweep (piecewise-deterministic Markov
    process) for trajectories ``traj_range``: reactions with ``continuous[j]``
    true form the flow, the others fire as jumps.

    Returns ``(out [S][N][T] float64, stats [T][4] uint64)`` with stats =
    (accepted steps, rejected steps and jump-location trials, jumps, status)."""
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    M, T = rates.shape
    cont = np.ascontiguousarray(np.asarray(continuous, dtype=bool).astype(np.int32))
    if cont.shape != (M,):
        raise ValueError("continuous must have one entry per reaction")
    a, b = traj_range if traj_range is not None else (0, T)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    times = np.ascontiguousarray(times, dtype=np.float64)
    S, N = len(times), net.n_species
    n = b - a
    out = np.zeros((S, N, n), dtype=np.float64)
    stats = np.zeros((n, 4), dtype=np.uint64)
    desc, keep = _desc(net)
    par = _HybridParams(int(seed), float(rtol), float(atol), int(max_steps))
    L = lib()
    nth = max(1, min(int(threads), n)) if n > 0 else 1
    bounds = np.linspace(0, n, nth + 1).astype(np.int64)

    def work(ci):
        lo, hi = int(bounds[ci]), int(bounds[ci + 1])
        if hi <= lo:
            return 0
        rp = rates.ctypes.data + 8 * (a + lo)
        if x0.ndim == 2:
            xp, xld = x0.ctypes.data + 4 * (a + lo), T
        else:
            xp, xld = x0.ctypes.data, 0
        return L.orc_hybrid_run(C.byref(desc), cont.ctypes.data, rp, T, xp, xld,
                                times.ctypes.data, S, a + lo, hi - lo, out.ctypes.data + 8 * lo,
                                n, stats.ctypes.data + 32 * lo, C.byref(par))

    if nth == 1:
        rcs = [work(0)]
    else:
        with ThreadPoolExecutor(nth) as ex:
            rcs = list(ex.map(work, range(nth)))
    for rc in rcs:
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}")
    del keep
    return out, stats
