"""Compile the HIP library in-tree for gfx950 (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpaper_rt.so")
SOURCES = ["csrc/rt_api.cpp", "csrc/rt_desc.cpp", "csrc/rt_geodesic.cpp", "csrc/rt_latlong.cpp", "csrc/rt_mapr.cpp", "csrc/rt_geometry.cpp",
           "csrc/k_step.hip", "csrc/k_march.hip", "csrc/k_column.hip", "csrc/k_adjoint.hip",
           "csrc/k_adj_march.hip", "csrc/k_adj_column.hip", "csrc/k_gas.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # reproducible face fluxes: the two cells sharing a face evaluate it with
    # identical arithmetic, so no contraction differences between call sites
    "-ffp-contract=off",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed (exit %d): %s" % (res.returncode, cmd[-1]))


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source to an object (in parallel), then link the shared
    library next to this file; the previous library is replaced atomically."""
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]
    jobs = jobs or min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="paper_rt_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [["hipcc"] + FLAGS + inc + ["-c", os.path.join(HERE, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", LIB + ".tmp"],
             verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
