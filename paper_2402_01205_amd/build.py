"""Builds libtpc.so (gfx950) in-tree with hipcc.

Flags: -ffp-contract=off keeps every FP32 expression exactly as written (no FMA
contraction), which the bit-exact parity with the CPU oracle relies on; HIP's
default correctly rounded FP32 division and square root are kept; packed FP32
instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", "tpc.hip")]
DEPS = SRC + [os.path.join(HERE, "csrc", f) for f in ("tpc_math.h", "tpc_kernels.h")] + [
    os.path.join(ROOT, "include", "tpc.h")]
LIB = os.path.join(HERE, "libtpc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("TPC_OFFLOAD_ARCH", "gfx950")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I" + os.path.join(ROOT, "include")]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in DEPS):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
    sys.exit(0)
