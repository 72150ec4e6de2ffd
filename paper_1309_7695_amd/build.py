"""Compile the HIP library (``librn.so``) for gfx950 in-tree with hipcc."""
import os
import subprocess
import sys

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
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-promote-alloca-to-vector-limit=4096",
         "-Wno-unused-command-line-argument"]


def sources():
    return [os.path.join(CSRC, "rn_host.cpp"), os.path.join(CSRC, "rn_sweep.hip"),
            os.path.join(CSRC, "rn_moments.hip"), os.path.join(CSRC, "rn_ode.hip")]


def build(verbose=False, extra=()):
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
