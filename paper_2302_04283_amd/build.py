"""Compile the HIP library in-tree for gfx950 (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpaper_rt.so")
SOURCES = ["csrc/rt_api.cpp", "csrc/rt_geodesic.cpp", "csrc/rt_geometry.cpp",
           "csrc/k_step.hip", "csrc/k_march.hip",
           "csrc/k_adjoint.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # reproducible face fluxes: the two cells sharing a face evaluate it with
    # identical arithmetic, so no contraction differences between call sites
    "-ffp-contract=off",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    cmd = (["hipcc"] + FLAGS + ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]
           + [os.path.join(HERE, s) for s in SOURCES] + ["-o", LIB + ".tmp"])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed (exit %d)" % res.returncode)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
