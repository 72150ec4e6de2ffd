"""The C ABI on the host: exported symbols, sample times, network validation
and argument checks that return before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1309_7695_amd import gen, rn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "rn.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rn_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    names = _header_functions()
    assert "rn_sweep" in names and "rn_load_network" in names and "rn_sample_times" in names
    L = rn.lib()
    for n in names:
        assert hasattr(L, n), n
    syms = subprocess.run(["nm", "-D", "--defined-only", rn.LIB_PATH], capture_output=True,
                          text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", syms, flags=re.M), n
    assert sorted(rn.EXPORTS) == names


def test_library_targets_gfx950(tmp_path):
    # the device code object bundled into the library is built for gfx950
    fb = tmp_path / "fatbin.bin"
    subprocess.run(["objcopy", f"--dump-section=.hip_fatbin={fb}", rn.LIB_PATH,
                    str(tmp_path / "copy.so")], check=True)
    data = fb.read_bytes()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


@pytest.mark.parametrize("t_end,n", [(100.0, 101), (50.0, 200), (10.0, 101), (1.0, 2), (3.0, 1),
                                      (0.3, 7)])
def test_sample_times_match_generator(t_end, n):
    got = rn.sample_times(t_end, n)
    want = gen.sample_times(t_end, n)
    assert np.array_equal(got, want)
    assert got[-1] == t_end
    if n > 1:
        assert got[0] == 0.0 and np.all(np.diff(got) > 0)


def test_sample_times_errors():
    L = rn.lib()
    buf = np.zeros(4)
    assert L.rn_sample_times(1.0, 0, buf.ctypes.data) == rn.RN_E_INVALID_ARG
    assert L.rn_sample_times(-1.0, 4, buf.ctypes.data) == rn.RN_E_INVALID_ARG
    assert L.rn_sample_times(float("nan"), 4, buf.ctypes.data) == rn.RN_E_INVALID_ARG
    assert L.rn_sample_times(float("inf"), 4, buf.ctypes.data) == rn.RN_E_INVALID_ARG
    assert L.rn_sample_times(1.0, 4, None) == rn.RN_E_INVALID_ARG


def _load(desc):
    h = C.c_void_p()
    return rn.lib().rn_load_network(C.byref(desc) if desc is not None else None, C.byref(h)), h


def _desc_from(n_species, reactions):
    net = gen.make_network(n_species, reactions)
    return rn.network_desc(net)


def test_load_network_validation():
    d, keep = _desc_from(2, [([(0, 1)], [(5, 1)])])        # product species out of range
    assert _load(d)[0] == rn.RN_E_INVALID_NETWORK
    d, keep = _desc_from(2, [([(-1, 1)], [])])              # negative species
    assert _load(d)[0] == rn.RN_E_INVALID_NETWORK
    d, keep = _desc_from(2, [([(0, 3)], [])])               # order 3
    assert _load(d)[0] == rn.RN_E_UNSUPPORTED
    d, keep = _desc_from(3, [([(0, 1), (1, 1), (2, 1)], [])])
    assert _load(d)[0] == rn.RN_E_UNSUPPORTED
    d, keep = _desc_from(2, [([(0, 0)], [])])               # zero coefficient
    assert _load(d)[0] == rn.RN_E_INVALID_NETWORK
    assert _load(None)[0] == rn.RN_E_INVALID_ARG
    d = rn.NetworkDesc(0, 1, None, None, None, None, None, None)
    assert _load(d)[0] == rn.RN_E_INVALID_ARG
    # offsets must not decrease
    rp = np.array([0, 1, 0], dtype=np.int32)
    sp = np.array([0], dtype=np.int32)
    co = np.array([1], dtype=np.int32)
    pp = np.array([0, 0, 0], dtype=np.int32)
    d = rn.NetworkDesc(1, 2, rp.ctypes.data, sp.ctypes.data, co.ctypes.data, pp.ctypes.data,
                       None, None)
    assert _load(d)[0] == rn.RN_E_INVALID_ARG


def test_load_valid_network_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    d, keep = rn.network_desc(gen.enzyme_network())
    rc, h = _load(d)
    assert rc == rn.RN_E_DEVICE
    assert not h.value


def test_sweep_argument_errors_are_synchronous():
    L = rn.lib()
    a = rn.SweepArgs()
    L.rn_sweep_args_init(C.byref(a))
    assert a.eps == 0.03 and a.n_c == 10 and a.ssa_factor == 10.0 and a.ssa_burst == 100
    assert a.max_steps == 10**8 and a.method == 0 and a.precision == 0
    assert L.rn_sweep(None, C.byref(a), None) == rn.RN_E_INVALID_ARG
    assert L.rn_strerror(rn.RN_E_UNSUPPORTED).startswith(b"unsupported")
    assert L.rn_strerror(12345) == b"unknown error"


def test_binding_refuses_host_tensors():
    import torch

    class Fake:
        n_species, n_reactions = 1, 1
    z = torch.zeros(1)
    with pytest.raises(ValueError):
        rn.sweep(Fake(), z, z, z, z, torch.zeros((1, 4), dtype=torch.int64), seed=1)


def test_precision_constants_match_header():
    import re
    text = open(os.path.join(ROOT, "include", "rn.h")).read()
    consts = dict(re.findall(r"#define (RN_FP\d\d) (\d+)", text))
    assert int(consts["RN_FP64"]) == rn.FP64 == rn.PRECISIONS["fp64"]
    assert int(consts["RN_FP32"]) == rn.FP32 == rn.PRECISIONS["fp32"]


def test_binding_refuses_unknown_precision():
    import torch
    z = torch.zeros(1)
    with pytest.raises(ValueError):
        rn.sweep(None, z, z, z, z, torch.zeros((1, 4), dtype=torch.int64), seed=1,
                 precision="fp16")


def test_batch_handle_without_device():
    L = rn.lib()
    h = C.c_void_p()
    assert L.rn_batch_create(C.byref(h)) == rn.RN_OK and h.value
    assert L.rn_batch_size(h) == 0
    assert L.rn_batch_launch(h, None) == rn.RN_OK  # nothing to launch
    a = rn.SweepArgs()
    L.rn_sweep_args_init(C.byref(a))
    assert L.rn_batch_add(h, None, C.byref(a)) == rn.RN_E_INVALID_ARG
    assert L.rn_batch_add(None, None, C.byref(a)) == rn.RN_E_INVALID_ARG
    assert L.rn_batch_create(None) == rn.RN_E_INVALID_ARG
    assert L.rn_batch_size(None) == rn.RN_E_INVALID_ARG
    L.rn_batch_free(h)
    L.rn_batch_free(None)


def test_server_argument_errors_without_device():
    L = rn.lib()
    h = C.c_void_p()
    assert L.rn_server_create(0, 1, C.byref(h)) == rn.RN_E_INVALID_ARG
    assert L.rn_server_create(1 << 20, 0, C.byref(h)) == rn.RN_E_INVALID_ARG
    assert L.rn_server_create(1 << 20, 1, None) == rn.RN_E_INVALID_ARG
    import torch
    if not torch.cuda.is_available():
        assert L.rn_server_create(1 << 20, 1, C.byref(h)) == rn.RN_E_DEVICE
    n = C.c_int32()
    assert L.rn_server_poll(None, None, 0, C.byref(n)) == rn.RN_E_INVALID_ARG
    assert L.rn_server_fetch(None, 1, None, None) == rn.RN_E_INVALID_ARG
    assert L.rn_server_submit(None, None, None) == rn.RN_E_INVALID_ARG
    L.rn_server_free(None)


def test_hybrid_args_defaults_and_host_checks():
    L = rn.lib()
    a = rn.HybridArgs()
    L.rn_hybrid_args_init(C.byref(a))
    assert (a.rtol, a.atol, a.max_steps, a.seed, a.traj_offset) == (1e-6, 1e-6, 10**7, 0, 0)
    assert L.rn_hybrid_work_doubles(None, 10) == -1
    assert L.rn_hybrid_sweep(None, C.byref(a), None) == rn.RN_E_INVALID_ARG
    # argument checks that return before any device call (no network needed)
    a.n_times = 0
    assert L.rn_hybrid_sweep(None, C.byref(a), None) == rn.RN_E_INVALID_ARG
