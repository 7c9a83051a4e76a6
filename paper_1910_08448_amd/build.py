"""Builds libmpr.so (the HIP library behind include/mpr.h) in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmpr.so")
SOURCES = [os.path.join(CSRC, "mpr.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("mpr_device.hpp", "mpr_sparse.hpp", "mpr_tiled.hpp")] + [
    os.path.join(ROOT, "include", "mpr.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit FMA contraction: every fused multiply-add in the kernels is written out, so
    # all kernel variants round identically
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function", "-Wno-bitwise-instead-of-logical",
]


def hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def build(verbose=False):
    """Compiles the library every time it is called (the output is replaced atomically)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
