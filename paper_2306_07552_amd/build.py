"""Builds libgal.so (hipcc, gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libgal.so")

SOURCES = ["gal_api.cpp", "gal_mlp_api.cpp", "k_robot.hip", "k_grid.hip", "k_raster.hip",
           "k_util.hip", "k_mlp.hip", "k_surrogate.hip", "k_sur_infer.hip",
           "gal_noalloc.cpp", "k_policy.hip", "gal_policy_api.cpp"]

# Exact binary32 semantics on the device: no contraction into FMA, correctly
# rounded division and square root, denormals kept; packed-FP32 instructions
# disabled.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-x", "hip",
            "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = True) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = (["/opt/rocm/bin/hipcc"] + HIPFLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", LIB + ".tmp"] + srcs)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
