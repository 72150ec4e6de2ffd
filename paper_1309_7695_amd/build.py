"""Compile the HIP library (``librn.so``) for gfx950 in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librn.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: every floating-point operation is rounded once, in the
# written order (no fused multiply-add), as the method's arithmetic is specified.
# -packed-fp32-ops: no packed FP32 instructions are generated.
# promote-alloca-to-vector-limit: lets the per-lane rate vectors (up to 8 x 16
# doubles) stay in VGPRs instead of being demoted to scratch memory.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-promote-alloca-to-vector-limit=4096",
         "-Wno-unused-command-line-argument"]


def sources():
    return [os.path.join(CSRC, f) for f in
            ("rn_host.cpp", "rn_sweep_f64.hip", "rn_sweep_f32.hip", "rn_moments.hip",
             "rn_ode.hip")]


def build(verbose=False, extra=(), jobs=None):
    """Compile each source to an object (in parallel), then link librn.so."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, *extra, *inc, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    srcs = sources()
    with ThreadPoolExecutor(max_workers=jobs or min(len(srcs), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
