"""ctypes binding of the C ABI in ``include/rn.h`` (``librn.so``).

Argument marshalling only: every step of the simulation runs in the library's
HIP kernels.  PyTorch supplies device memory and the HIP stream.  When the
library has not been built this module raises instead of falling back to
anything else.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librn.so")

RN_OK = 0
RN_E_INVALID_ARG = -1
RN_E_INVALID_NETWORK = -2
RN_E_UNSUPPORTED = -3
RN_E_NOMEM = -4
RN_E_DEVICE = -5
RN_E_SCRATCH = -6
ST_ABSORBED, ST_MAXSTEPS, ST_OVERFLOW = 1, 2, 4
METHOD_TAULEAP, METHOD_SSA = 0, 1
OUT_SAMPLE_MAJOR, OUT_TRAJ_MAJOR = 0, 1
LAYOUTS = {"sample": OUT_SAMPLE_MAJOR, "traj": OUT_TRAJ_MAJOR}
FP64, FP32 = 0, 1
PRECISIONS = {"fp64": FP64, "fp32": FP32}

EXPORTS = ["rn_load_network", "rn_free_network", "rn_network_species", "rn_network_reactions",
           "rn_sample_times", "rn_sweep_args_init", "rn_sweep", "rn_sweep_kernel_kind", "rn_compile_drain",
           "rn_batch_create", "rn_batch_persistent", "rn_batch_tune", "rn_batch_add",
           "rn_batch_size", "rn_batch_launch", "rn_batch_free",
           "rn_server_create", "rn_server_submit", "rn_server_poll", "rn_server_fetch",
           "rn_server_status", "rn_server_free",
           "rn_moments", "rn_ode_args_init",
           "rn_ode_work_doubles", "rn_ode_sweep", "rn_ode_sweep_noalloc",
           "rn_ode_noalloc_max_traj", "rn_hybrid_args_init", "rn_hybrid_work_doubles",
           "rn_hybrid_sweep", "rn_strerror", "rn_last_device_error"]


class NetworkDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("react_ptr", C.c_void_p), ("react_species", C.c_void_p),
                ("react_coeff", C.c_void_p), ("prod_ptr", C.c_void_p),
                ("prod_species", C.c_void_p), ("prod_coeff", C.c_void_p)]


class SweepArgs(C.Structure):
    _fields_ = [("n_traj", C.c_int64), ("traj_offset", C.c_int64),
                ("rates", C.c_void_p), ("rates_ld", C.c_int64),
                ("x0", C.c_void_p), ("x0_ld", C.c_int64),
                ("times", C.c_void_p), ("n_times", C.c_int32),
                ("out", C.c_void_p), ("out_ld", C.c_int64),
                ("stats", C.c_void_p), ("seed", C.c_uint64),
                ("eps", C.c_double), ("n_c", C.c_int32), ("ssa_factor", C.c_double),
                ("ssa_burst", C.c_int32), ("max_steps", C.c_uint64),
                ("method", C.c_int32), ("precision", C.c_int32), ("cle_threshold", C.c_double),
                ("phase_cycles", C.c_void_p), ("sum_x", C.c_void_p), ("sum_x2", C.c_void_p),
                ("hist", C.c_void_p), ("hist_lo", C.c_void_p), ("hist_width", C.c_void_p),
                ("hist_bins", C.c_int32), ("out_layout", C.c_int32)]


class ServeJob(C.Structure):
    _fields_ = [("net", C.c_void_p), ("n_traj", C.c_int64), ("rates", C.c_void_p),
                ("x0", C.c_void_p), ("x0_per_traj", C.c_int32), ("times", C.c_void_p),
                ("n_times", C.c_int32), ("params", SweepArgs)]


class OdeArgs(C.Structure):
    _fields_ = [("n_traj", C.c_int64), ("rates", C.c_void_p), ("rates_ld", C.c_int64),
                ("x0", C.c_void_p), ("x0_ld", C.c_int64), ("times", C.c_void_p),
                ("n_times", C.c_int32), ("out", C.c_void_p), ("out_ld", C.c_int64),
                ("stats", C.c_void_p), ("work", C.c_void_p), ("work_ld", C.c_int64),
                ("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_uint64),
                ("method", C.c_int32)]


ODE_METHODS = {"dopri5": 0, "ros4": 1}


class HybridArgs(C.Structure):
    _fields_ = [("n_traj", C.c_int64), ("traj_offset", C.c_int64), ("continuous", C.c_void_p),
                ("rates", C.c_void_p), ("rates_ld", C.c_int64), ("x0", C.c_void_p),
                ("x0_ld", C.c_int64), ("times", C.c_void_p), ("n_times", C.c_int32),
                ("out", C.c_void_p), ("out_ld", C.c_int64), ("stats", C.c_void_p),
                ("work", C.c_void_p), ("work_ld", C.c_int64), ("seed", C.c_uint64),
                ("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_uint64)]


class RNError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().rn_strerror(code).decode()
        if code == RN_E_DEVICE:
            msg += f" (hipError {lib().rn_last_device_error()})"
        super().__init__(f"{what}: {msg} [{code}]" if what else f"{msg} [{code}]")


_lib = None


def _torch_device_first():
    """Initialise torch's device state before the library makes its first HIP
    call: torch initialised only after one of the library's run-time kernel
    compiles has been seen to report no device."""
    import torch
    if torch.cuda.device_count() > 0:
        torch.cuda.init()


def lib():
    """Load ``librn.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1309_7695_amd.build`")
        _torch_device_first()
        L = C.CDLL(LIB_PATH)
        L.rn_load_network.argtypes = [C.POINTER(NetworkDesc), C.POINTER(C.c_void_p)]
        L.rn_load_network.restype = C.c_int
        L.rn_free_network.argtypes = [C.c_void_p]
        L.rn_free_network.restype = None
        L.rn_network_species.argtypes = [C.c_void_p]
        L.rn_network_species.restype = C.c_int32
        L.rn_network_reactions.argtypes = [C.c_void_p]
        L.rn_network_reactions.restype = C.c_int32
        L.rn_sample_times.argtypes = [C.c_double, C.c_int32, C.c_void_p]
        L.rn_sample_times.restype = C.c_int
        L.rn_sweep_args_init.argtypes = [C.POINTER(SweepArgs)]
        L.rn_sweep_args_init.restype = None
        L.rn_sweep.argtypes = [C.c_void_p, C.POINTER(SweepArgs), C.c_void_p]
        L.rn_sweep.restype = C.c_int
        L.rn_sweep_kernel_kind.argtypes = [C.c_void_p, C.c_int32, C.c_int64]
        L.rn_sweep_kernel_kind.restype = C.c_int
        L.rn_compile_drain.argtypes = []
        L.rn_compile_drain.restype = None
        L.rn_batch_create.argtypes = [C.POINTER(C.c_void_p)]
        L.rn_batch_create.restype = C.c_int
        L.rn_batch_persistent.argtypes = [C.c_void_p, C.c_int32]
        L.rn_batch_persistent.restype = C.c_int
        L.rn_batch_tune.argtypes = [C.c_void_p, C.c_void_p]
        L.rn_batch_tune.restype = C.c_int
        L.rn_batch_add.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(SweepArgs)]
        L.rn_batch_add.restype = C.c_int
        L.rn_batch_size.argtypes = [C.c_void_p]
        L.rn_batch_size.restype = C.c_int
        L.rn_batch_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.rn_batch_launch.restype = C.c_int
        L.rn_batch_free.argtypes = [C.c_void_p]
        L.rn_batch_free.restype = None
        L.rn_server_create.argtypes = [C.c_int64, C.c_int32, C.POINTER(C.c_void_p)]
        L.rn_server_create.restype = C.c_int
        L.rn_server_submit.argtypes = [C.c_void_p, C.POINTER(ServeJob), C.POINTER(C.c_int64)]
        L.rn_server_submit.restype = C.c_int
        L.rn_server_poll.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
        L.rn_server_poll.restype = C.c_int
        L.rn_server_fetch.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.rn_server_fetch.restype = C.c_int
        L.rn_server_status.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64)]
        L.rn_server_status.restype = C.c_int
        L.rn_server_free.argtypes = [C.c_void_p]
        L.rn_server_free.restype = None
        L.rn_moments.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int64,
                                 C.c_void_p, C.c_void_p, C.c_void_p]
        L.rn_moments.restype = C.c_int
        L.rn_ode_args_init.argtypes = [C.POINTER(OdeArgs)]
        L.rn_ode_args_init.restype = None
        L.rn_ode_work_doubles.argtypes = [C.c_void_p, C.c_int64]
        L.rn_ode_work_doubles.restype = C.c_int64
        L.rn_ode_sweep.argtypes = [C.c_void_p, C.POINTER(OdeArgs), C.c_void_p]
        L.rn_ode_sweep.restype = C.c_int
        L.rn_ode_sweep_noalloc.argtypes = [C.c_void_p, C.POINTER(OdeArgs), C.c_void_p]
        L.rn_ode_sweep_noalloc.restype = C.c_int
        L.rn_ode_noalloc_max_traj.argtypes = [C.c_void_p]
        L.rn_ode_noalloc_max_traj.restype = C.c_int64
        L.rn_hybrid_args_init.argtypes = [C.POINTER(HybridArgs)]
        L.rn_hybrid_args_init.restype = None
        L.rn_hybrid_work_doubles.argtypes = [C.c_void_p, C.c_int64]
        L.rn_hybrid_work_doubles.restype = C.c_int64
        L.rn_hybrid_sweep.argtypes = [C.c_void_p, C.POINTER(HybridArgs), C.c_void_p]
        L.rn_hybrid_sweep.restype = C.c_int
        L.rn_strerror.argtypes = [C.c_int]
        L.rn_strerror.restype = C.c_char_p
        L.rn_last_device_error.argtypes = []
        L.rn_last_device_error.restype = C.c_int
        _lib = L
        # background compilations end before the interpreter tears down
        atexit.register(L.rn_compile_drain)
    return _lib


def _check(rc, what):
    if rc != RN_OK:
        raise RNError(rc, what)


def sample_times(t_end, n_points):
    out = np.zeros(max(int(n_points), 1), dtype=np.float64)
    _check(lib().rn_sample_times(float(t_end), int(n_points), out.ctypes.data), "rn_sample_times")
    return out


def network_desc(net):
    """(NetworkDesc, keep-alive arrays) for a ``gen.Network``-like object or a
    dict of CSR arrays plus ``n_species``."""
    if isinstance(net, dict):
        arrs = {k: np.ascontiguousarray(net[k], dtype=np.int32) for k in
                ("react_ptr", "react_species", "react_coeff", "prod_ptr", "prod_species",
                 "prod_coeff")}
        ns = int(net["n_species"])
    else:
        arrs = {k: np.ascontiguousarray(v, dtype=np.int32) for k, v in net.csr().items()}
        ns = int(net.n_species)
    nr = len(arrs["react_ptr"]) - 1
    d = NetworkDesc(ns, nr, *(arrs[k].ctypes.data if arrs[k].size else None for k in
                              ("react_ptr", "react_species", "react_coeff", "prod_ptr",
                               "prod_species", "prod_coeff")))
    return d, arrs


class Network:
    """A network loaded onto the current HIP device (``rn_load_network``)."""

    def __init__(self, net):
        d, keep = network_desc(net)
        h = C.c_void_p()
        _check(lib().rn_load_network(C.byref(d), C.byref(h)), "rn_load_network")
        self._h = h
        self.n_species = lib().rn_network_species(h)
        self.n_reactions = lib().rn_network_reactions(h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().rn_free_network(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sweep_args(net: Network, rates, x0, times, out, stats, *, seed, traj_offset=0, eps=0.03,
               n_c=10, ssa_factor=10.0, ssa_burst=100, max_steps=10**8, method=METHOD_TAULEAP,
               cle_threshold=0.0, precision="fp64", phase_cycles=None, sum_x=None, sum_x2=None,
               hist=None, hist_lo=None, hist_width=None, out_layout="sample"):
    """Check the tensors and marshal an ``rn_sweep_args`` for them.

    ``rates`` float64 [M][>=T] (row stride = ld), ``x0`` int32 [N] or [N][>=T],
    ``times`` float64 [S], ``out`` int32 [S][N][>=T] (last dim stride = ld) or
    None when fused statistics are asked for, ``stats`` uint64/int64 [T][4]; all
    CUDA (HIP) tensors on the network's device.  T is taken from ``stats``.
    ``precision`` is "fp64" or "fp32" (RN_FP64 / RN_FP32).  Fused statistics:
    ``sum_x`` 64-bit [S][N] with ``sum_x2`` 64-bit [S][N][2] (exact sums of x and
    x^2, the latter as 128-bit low/high words), ``hist`` int32 [S][N][B] with
    ``hist_lo`` and ``hist_width`` int32 [N] (bin edges per species).
    ``out_layout="traj"`` takes ``out`` as int32 [>=T][S][N] (each trajectory's
    samples contiguous) instead of [S][N][>=T]."""
    import torch

    if precision not in PRECISIONS:
        raise ValueError("precision must be 'fp64' or 'fp32'")
    T = int(stats.shape[0])
    for name, t in (("rates", rates), ("x0", x0), ("times", times), ("out", out),
                    ("stats", stats), ("sum_x", sum_x), ("sum_x2", sum_x2), ("hist", hist),
                    ("hist_lo", hist_lo), ("hist_width", hist_width)):
        if t is not None and not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
    if out is None and sum_x is None and hist is None:
        raise ValueError("out may be None only when sum_x or hist is given")
    if rates.dtype != torch.float64 or times.dtype != torch.float64:
        raise TypeError("rates and times must be float64")
    if x0.dtype != torch.int32 or (out is not None and out.dtype != torch.int32):
        raise TypeError("x0 and out must be int32")
    if stats.dtype not in (torch.int64, torch.uint64) or tuple(stats.shape) != (T, 4) or \
            not stats.is_contiguous():
        raise TypeError("stats must be a contiguous 64-bit [T][4] tensor")
    if rates.dim() != 2 or rates.stride(1) != 1 or rates.shape[0] != net.n_reactions:
        raise ValueError("rates must be [M][T] with unit trajectory stride")
    if out_layout not in LAYOUTS:
        raise ValueError("out_layout must be 'sample' or 'traj'")
    traj_major = out_layout == "traj"
    if out is not None and not traj_major and (
            out.dim() != 3 or out.stride(2) != 1 or out.shape[1] != net.n_species or
            out.stride(0) != out.shape[1] * out.stride(1) or out.shape[0] != times.numel()):
        raise ValueError("out must be [S][N][T] with unit trajectory stride")
    if out is not None and traj_major and (
            out.dim() != 3 or out.shape[1] != times.numel() or out.shape[2] != net.n_species or
            out.stride(2) != 1 or out.stride(1) != net.n_species):
        raise ValueError("out must be [T][S][N] with contiguous [S][N] rows")
    if not times.is_contiguous():
        raise ValueError("times must be contiguous")
    if rates.shape[1] < T or (out is not None and out.shape[0 if traj_major else 2] < T):
        raise ValueError("rates and out need at least one column per trajectory")
    S, N = times.numel(), net.n_species
    if (sum_x is None) != (sum_x2 is None):
        raise ValueError("sum_x and sum_x2 go together")
    if sum_x is not None:
        if sum_x.dtype not in (torch.int64, torch.uint64) or sum_x.numel() != S * N or \
                not sum_x.is_contiguous() or sum_x2.dtype not in (torch.int64, torch.uint64) or \
                sum_x2.numel() != 2 * S * N or not sum_x2.is_contiguous():
            raise ValueError("sum_x must be 64-bit [S][N] and sum_x2 64-bit [S][N][2], contiguous")
    bins = 0
    if hist is not None:
        if hist.dtype != torch.int32 or hist.numel() % (S * N) != 0 or not hist.is_contiguous():
            raise ValueError("hist must be a contiguous int32 [S][N][B] tensor")
        bins = hist.numel() // (S * N)
        for name, t in (("hist_lo", hist_lo), ("hist_width", hist_width)):
            if t is None or t.dtype != torch.int32 or t.numel() != N or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous int32 [N] device tensor")
    if x0.dim() == 1:
        x0_ld = 0
        if x0.numel() != net.n_species or not x0.is_contiguous():
            raise ValueError("x0 must have one entry per species")
    else:
        if x0.stride(1) != 1 or x0.shape[0] != net.n_species or x0.shape[1] < T:
            raise ValueError("per-trajectory x0 must be [N][T] with unit trajectory stride")
        x0_ld = x0.stride(0)
    a = SweepArgs()
    lib().rn_sweep_args_init(C.byref(a))
    a.n_traj = T
    a.traj_offset = int(traj_offset)
    a.rates, a.rates_ld = rates.data_ptr(), rates.stride(0)
    a.x0, a.x0_ld = x0.data_ptr(), x0_ld
    a.times, a.n_times = times.data_ptr(), times.numel()
    a.out_layout = LAYOUTS[out_layout]
    if out is not None:
        a.out, a.out_ld = out.data_ptr(), (out.stride(0) if traj_major else out.stride(1))
    a.stats = stats.data_ptr()
    if sum_x is not None:
        a.sum_x, a.sum_x2 = sum_x.data_ptr(), sum_x2.data_ptr()
    if hist is not None:
        a.hist, a.hist_bins = hist.data_ptr(), bins
        a.hist_lo, a.hist_width = hist_lo.data_ptr(), hist_width.data_ptr()
    a.seed = int(seed) & (2**64 - 1)
    a.eps, a.n_c, a.ssa_factor = float(eps), int(n_c), float(ssa_factor)
    a.ssa_burst, a.max_steps, a.method, a.precision = int(ssa_burst), int(max_steps), \
        int(method), PRECISIONS[precision]
    a.cle_threshold = float(cle_threshold)
    if phase_cycles is not None:
        if not phase_cycles.is_cuda or phase_cycles.dtype not in (torch.int64, torch.uint64) or \
                phase_cycles.numel() < 4 * ((T + 63) // 64) or not phase_cycles.is_contiguous():
            raise ValueError("phase_cycles must be a contiguous 64-bit device tensor "
                             "of at least 4 * ceil(T / 64) entries")
        a.phase_cycles = phase_cycles.data_ptr()
    return a


def sweep(net: Network, rates, x0, times, out, stats, *, stream=None, **kw):
    """Enqueue ``rn_sweep`` on ``stream`` (default: torch's current stream); the
    arguments are those of ``sweep_args``.  Returns immediately."""
    import torch

    a = sweep_args(net, rates, x0, times, out, stats, **kw)
    if stream is None:
        stream = torch.cuda.current_stream(rates.device)
    _check(lib().rn_sweep(net.handle, C.byref(a), C.c_void_p(stream.cuda_stream)), "rn_sweep")


class Batch:
    """``rn_batch``: sweep jobs launched together through one HIP graph.

    ``add`` takes the arguments of ``sweep``; the batch keeps the tensors and
    networks alive.  The first ``launch`` records the graph, later ones replay
    it (rewriting the same output tensors)."""

    def __init__(self, persistent=False):
        h = C.c_void_p()
        _check(lib().rn_batch_create(C.byref(h)), "rn_batch_create")
        self.handle = h
        self._keep = []
        if persistent:
            _check(lib().rn_batch_persistent(self.handle, 1), "rn_batch_persistent")

    def add(self, net: Network, rates, x0, times, out, stats, **kw):
        a = sweep_args(net, rates, x0, times, out, stats, **kw)
        _check(lib().rn_batch_add(self.handle, net.handle, C.byref(a)), "rn_batch_add")
        self._keep.append((net, rates, x0, times, out, stats, kw))

    def tune(self, stream=None):
        """``rn_batch_tune``: time the persistent form's launch shapes per bucket."""
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().rn_batch_tune(self.handle, C.c_void_p(stream.cuda_stream)), "rn_batch_tune")

    def __len__(self):
        n = lib().rn_batch_size(self.handle)
        if n < 0:
            raise RNError(n, "rn_batch_size")
        return n

    def launch(self, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().rn_batch_launch(self.handle, C.c_void_p(stream.cuda_stream)),
               "rn_batch_launch")

    def close(self):
        if self.handle:
            lib().rn_batch_free(self.handle)
            self.handle = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sweep_kernel_kind(net: Network, n_traj, precision="fp64"):
    """``rn_sweep_kernel_kind``: "network" when rn_sweep runs a kernel compiled
    for this network (compiling it now if needed), "wave" for the generic
    one-wave-per-trajectory kernel, "generic" for the generic
    one-lane-per-trajectory kernel."""
    if precision not in PRECISIONS:
        raise ValueError("precision must be 'fp64' or 'fp32'")
    rc = lib().rn_sweep_kernel_kind(net.handle, PRECISIONS[precision], int(n_traj))
    if rc < 0:
        raise RNError(rc, "rn_sweep_kernel_kind")
    return {1: "network", 2: "wave"}.get(rc, "generic")


class Server:
    """``rn_server``: sweep jobs admitted continuously into an HBM budget.

    ``submit(net, rates, x0, times, seed=..., **options)`` takes host (numpy)
    arrays and returns a job id; ``poll()`` advances the server and returns the
    ids that finished; ``fetch(id)`` returns ``(out [S][N][T] int32, stats
    [T][4] uint64)`` and frees the job's memory."""

    def __init__(self, budget_bytes, max_running=4):
        h = C.c_void_p()
        _check(lib().rn_server_create(int(budget_bytes), int(max_running), C.byref(h)),
               "rn_server_create")
        self.handle = h
        self._jobs = {}

    def submit(self, net: Network, rates, x0, times, *, seed, eps=0.03, n_c=10,
               ssa_factor=10.0, ssa_burst=100, max_steps=10**8, method=METHOD_TAULEAP,
               cle_threshold=0.0, precision="fp64"):
        rates = np.ascontiguousarray(rates, dtype=np.float64)
        x0 = np.ascontiguousarray(x0, dtype=np.int32)
        times = validate_times(times)
        M, T = rates.shape
        if M != net.n_reactions or x0.shape[0] != net.n_species or \
                (x0.ndim == 2 and x0.shape[1] != T):
            raise ValueError("rates must be [M][T], x0 [N] or [N][T]")
        if precision not in PRECISIONS:
            raise ValueError("precision must be 'fp64' or 'fp32'")
        j = ServeJob()
        j.net, j.n_traj = net.handle.value, T
        j.rates, j.x0, j.x0_per_traj = rates.ctypes.data, x0.ctypes.data, int(x0.ndim == 2)
        j.times, j.n_times = times.ctypes.data, len(times)
        lib().rn_sweep_args_init(C.byref(j.params))
        p = j.params
        p.seed = int(seed) & (2**64 - 1)
        p.eps, p.n_c, p.ssa_factor = float(eps), int(n_c), float(ssa_factor)
        p.ssa_burst, p.max_steps, p.method = int(ssa_burst), int(max_steps), int(method)
        p.precision, p.cle_threshold = PRECISIONS[precision], float(cle_threshold)
        jid = C.c_int64()
        _check(lib().rn_server_submit(self.handle, C.byref(j), C.byref(jid)), "rn_server_submit")
        self._jobs[jid.value] = (net, len(times), net.n_species, T)
        return jid.value

    def poll(self, max_ids=1024):
        ids = np.zeros(max_ids, dtype=np.int64)
        n = C.c_int32()
        _check(lib().rn_server_poll(self.handle, ids.ctypes.data, int(max_ids), C.byref(n)),
               "rn_server_poll")
        return [int(v) for v in ids[:n.value]]

    def fetch(self, job_id):
        net, S, N, T = self._jobs[job_id]
        out = np.empty((S, N, T), dtype=np.int32)
        st = np.empty((T, 4), dtype=np.uint64)
        _check(lib().rn_server_fetch(self.handle, int(job_id), out.ctypes.data, st.ctypes.data),
               "rn_server_fetch")
        del self._jobs[job_id]
        return out, st

    def status(self):
        q, r, b = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().rn_server_status(self.handle, C.byref(q), C.byref(r), C.byref(b)),
               "rn_server_status")
        return {"queued": q.value, "running": r.value, "bytes_in_use": b.value}

    def close(self):
        if self.handle:
            lib().rn_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def precompile(nets, n_traj, precision="fp64", threads=8):
    """Compile the kernels of several networks concurrently (the library lets
    different networks compile in parallel; ctypes releases the GIL).  Returns
    the kernel kinds, in order."""
    from concurrent.futures import ThreadPoolExecutor

    n_traj = list(n_traj) if hasattr(n_traj, "__len__") else [n_traj] * len(nets)
    with ThreadPoolExecutor(max_workers=max(1, int(threads))) as ex:
        return list(ex.map(lambda a: sweep_kernel_kind(a[0], a[1], precision),
                           zip(nets, n_traj)))


def validate_times(times):
    t = np.asarray(times, dtype=np.float64)
    if t.ndim != 1 or t.size < 1 or not np.all(np.isfinite(t)) or np.any(t < 0) or \
            np.any(np.diff(t) <= 0):
        raise ValueError("times must be finite, non-negative and strictly increasing")
    return t


def run(net_desc, rates, x0, times, *, seed, device="cuda", method="tauleap", **kw):
    """Host-array convenience: upload, sweep, synchronize, download.

    Returns ``(out [S][N][T] int32, stats [T][4] uint64)`` as numpy arrays."""
    import torch

    times = validate_times(times)
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    M, T = rates.shape
    dev = torch.device(device)
    net = net_desc if isinstance(net_desc, Network) else Network(net_desc)
    S, N = len(times), net.n_species
    r_d = torch.from_numpy(rates).to(dev)
    x_d = torch.from_numpy(x0).to(dev)
    t_d = torch.from_numpy(times).to(dev)
    o_d = torch.empty((S, N, T), dtype=torch.int32, device=dev)
    s_d = torch.empty((T, 4), dtype=torch.int64, device=dev)
    sweep(net, r_d, x_d, t_d, o_d, s_d, seed=seed,
          method=METHOD_SSA if method == "ssa" else METHOD_TAULEAP, **kw)
    torch.cuda.synchronize(dev)
    return o_d.cpu().numpy(), s_d.cpu().numpy().view(np.uint64)


def moments(out, n_traj=None, *, sum_x=None, sum_x2=None, stream=None):
    """Enqueue ``rn_moments`` on the [S][N][>=T] int32 device tensor ``out``.

    Returns the device tensors ``(sum_x [S][N] int64, sum_x2 [S][N][2] int64
    holding the unsigned 128-bit low/high words)``; see :func:`moment_stats`."""
    import torch

    if not out.is_cuda or out.dtype != torch.int32 or out.dim() != 3 or out.stride(2) != 1 or \
            out.stride(0) != out.shape[1] * out.stride(1):
        raise ValueError("out must be a [S][N][T] int32 device tensor with unit trajectory stride")
    S, N = int(out.shape[0]), int(out.shape[1])
    T = int(out.shape[2]) if n_traj is None else int(n_traj)
    if sum_x is None:
        sum_x = torch.empty((S, N), dtype=torch.int64, device=out.device)
    if sum_x2 is None:
        sum_x2 = torch.empty((S, N, 2), dtype=torch.int64, device=out.device)
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    _check(lib().rn_moments(out.data_ptr(), out.stride(1), S, N, T, sum_x.data_ptr(),
                            sum_x2.data_ptr(), C.c_void_p(stream.cuda_stream)), "rn_moments")
    return sum_x, sum_x2


def moment_stats(sum_x, sum_x2, n_traj):
    """Exact host-side mean and unbiased variance from the integer sums."""
    sx = np.asarray(sum_x, dtype=np.int64)
    w = np.asarray(sum_x2, dtype=np.int64).view(np.uint64)
    s2 = [int(lo) + (int(hi) << 64) for lo, hi in zip(w[..., 0].ravel(), w[..., 1].ravel())]
    T = int(n_traj)
    mean = sx.astype(np.float64) / T
    var = np.array([(q - int(a) * int(a) / T) / (T - 1) if T > 1 else 0.0
                    for q, a in zip(s2, sx.ravel())]).reshape(sx.shape)
    return mean, var, np.array(s2, dtype=object).reshape(sx.shape)


def ode_sweep(net: Network, rates, x0, times, out, stats, work, *, rtol=1e-6, atol=1e-6,
              max_steps=10**7, method="dopri5", stream=None):
    """Enqueue ``rn_ode_sweep``: ``out`` float64 [S][N][>=T], ``work`` float64 device
    tensor of at least ``rn_ode_work_doubles`` elements; T from ``stats``.  With
    ``work=None`` it enqueues ``rn_ode_sweep_noalloc`` instead (the library's
    fixed scratch, at most ``rn_ode_noalloc_max_traj`` trajectories)."""
    import torch

    T = int(stats.shape[0])
    if out.dtype != torch.float64:
        raise TypeError("out must be float64")
    if work is not None:
        if work.dtype != torch.float64 or not work.is_contiguous():
            raise TypeError("work must be contiguous float64")
        if work.numel() < lib().rn_ode_work_doubles(net.handle, T):
            raise ValueError("work is too small")
    if rates.dim() != 2 or rates.stride(1) != 1 or out.dim() != 3 or out.stride(2) != 1 or \
            out.stride(0) != out.shape[1] * out.stride(1) or out.shape[0] != times.numel():
        raise ValueError("rates [M][T] and out [S][N][T] need unit trajectory stride")
    a = OdeArgs()
    lib().rn_ode_args_init(C.byref(a))
    a.n_traj = T
    a.rates, a.rates_ld = rates.data_ptr(), rates.stride(0)
    a.x0, a.x0_ld = x0.data_ptr(), (0 if x0.dim() == 1 else x0.stride(0))
    a.times, a.n_times = times.data_ptr(), times.numel()
    a.out, a.out_ld = out.data_ptr(), out.stride(1)
    a.stats = stats.data_ptr()
    if work is not None:
        a.work, a.work_ld = work.data_ptr(), T
    a.rtol, a.atol, a.max_steps = float(rtol), float(atol), int(max_steps)
    if method not in ODE_METHODS:
        raise ValueError("method must be 'dopri5' or 'ros4'")
    a.method = ODE_METHODS[method]
    if stream is None:
        stream = torch.cuda.current_stream(rates.device)
    if work is None:
        _check(lib().rn_ode_sweep_noalloc(net.handle, C.byref(a), C.c_void_p(stream.cuda_stream)),
               "rn_ode_sweep_noalloc")
    else:
        _check(lib().rn_ode_sweep(net.handle, C.byref(a), C.c_void_p(stream.cuda_stream)),
               "rn_ode_sweep")


def ode_run(net_desc, rates, x0, times, *, device="cuda", **kw):
    """Host-array convenience for :func:`ode_sweep`; returns numpy (out, stats)."""
    import torch

    times = validate_times(times)
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    M, T = rates.shape
    dev = torch.device(device)
    net = net_desc if isinstance(net_desc, Network) else Network(net_desc)
    S, N = len(times), net.n_species
    o = torch.empty((S, N, T), dtype=torch.float64, device=dev)
    s = torch.empty((T, 4), dtype=torch.int64, device=dev)
    work = torch.empty(max(lib().rn_ode_work_doubles(net.handle, T), 1), dtype=torch.float64,
                       device=dev)
    ode_sweep(net, torch.from_numpy(rates).to(dev), torch.from_numpy(x0).to(dev),
              torch.from_numpy(times).to(dev), o, s, work, **kw)
    torch.cuda.synchronize(dev)
    return o.cpu().numpy(), s.cpu().numpy().view(np.uint64)


def hybrid_sweep(net: Network, continuous, rates, x0, times, out, stats, work, *, seed,
                 rtol=1e-6, atol=1e-6, max_steps=10**7, traj_offset=0, stream=None):
    """Enqueue ``rn_hybrid_sweep``: ``continuous`` int32 device [M] (nonzero =
    continuous), ``out`` float64 [S][N][>=T], ``work`` float64 device tensor of at
    least ``rn_hybrid_work_doubles`` elements; T from ``stats``."""
    import torch

    T = int(stats.shape[0])
    if out.dtype != torch.float64 or work.dtype != torch.float64 or not work.is_contiguous():
        raise TypeError("out and work must be float64 (work contiguous)")
    if continuous.dtype != torch.int32 or continuous.numel() != net.n_reactions or \
            not continuous.is_contiguous():
        raise ValueError("continuous must be a contiguous int32 tensor with one entry per reaction")
    if work.numel() < lib().rn_hybrid_work_doubles(net.handle, T):
        raise ValueError("work is too small")
    if rates.dim() != 2 or rates.stride(1) != 1 or out.dim() != 3 or out.stride(2) != 1 or \
            out.stride(0) != out.shape[1] * out.stride(1) or out.shape[0] != times.numel():
        raise ValueError("rates [M][T] and out [S][N][T] need unit trajectory stride")
    a = HybridArgs()
    lib().rn_hybrid_args_init(C.byref(a))
    a.n_traj, a.traj_offset = T, int(traj_offset)
    a.continuous = continuous.data_ptr()
    a.rates, a.rates_ld = rates.data_ptr(), rates.stride(0)
    a.x0, a.x0_ld = x0.data_ptr(), (0 if x0.dim() == 1 else x0.stride(0))
    a.times, a.n_times = times.data_ptr(), times.numel()
    a.out, a.out_ld = out.data_ptr(), out.stride(1)
    a.stats = stats.data_ptr()
    a.work, a.work_ld = work.data_ptr(), T
    a.seed = int(seed)
    a.rtol, a.atol, a.max_steps = float(rtol), float(atol), int(max_steps)
    if stream is None:
        stream = torch.cuda.current_stream(rates.device)
    _check(lib().rn_hybrid_sweep(net.handle, C.byref(a), C.c_void_p(stream.cuda_stream)),
           "rn_hybrid_sweep")


def hybrid_run(net_desc, continuous, rates, x0, times, *, seed, device="cuda", **kw):
    """Host-array convenience for :func:`hybrid_sweep`; returns numpy (out, stats)."""
    import torch

    times = validate_times(times)
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    cont = np.ascontiguousarray(np.asarray(continuous, dtype=bool).astype(np.int32))
    M, T = rates.shape
    dev = torch.device(device)
    net = net_desc if isinstance(net_desc, Network) else Network(net_desc)
    S, N = len(times), net.n_species
    o = torch.empty((S, N, T), dtype=torch.float64, device=dev)
    s = torch.empty((T, 4), dtype=torch.int64, device=dev)
    work = torch.empty(max(lib().rn_hybrid_work_doubles(net.handle, T), 1), dtype=torch.float64,
                       device=dev)
    hybrid_sweep(net, torch.from_numpy(cont).to(dev), torch.from_numpy(rates).to(dev),
                 torch.from_numpy(x0).to(dev), torch.from_numpy(times).to(dev), o, s, work,
                 seed=seed, **kw)
    torch.cuda.synchronize(dev)
    return o.cpu().numpy(), s.cpu().numpy().view(np.uint64)
