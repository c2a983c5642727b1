"""Build the gfx950 HIP library ``libfstat.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libfstat.so")
SOURCES = [os.path.join(PKG, "csrc", "fstat_api.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain scalar/float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fuse per source expression only, the same way in every
    # kernel that inlines a helper (the grouped and per-template paths give
    # the same bits)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function", "-fvisibility=hidden",
    "-I", os.path.join(ROOT, "include"),
]


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source into libfstat.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
