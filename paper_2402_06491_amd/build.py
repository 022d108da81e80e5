"""Build libbrt.so (HIP kernels + host runtime) for gfx950 with hipcc, in the package directory."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libbrt.so")
SOURCES = ["brt_kernels.hip", "brt_moments.hip", "brt_runtime.hip", "brt_serve.hip", "brt_tune.hip", "brt_pdd.hip",
           "brt_noalloc.hip"]
# Packed FP32 VALU forms are disabled for every HIP translation unit (the compiler would otherwise
# form v_pk_* from ordinary float code).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(PKG, "csrc", s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
