"""Build the MI355X library libidp.so in-tree (hipcc for gfx950, g++ host).

Device code is compiled without FMA contraction and without fast-math so
that every FP64 operation is a single IEEE-rounded add, sub, mul, div or
sqrt in source order (explicit fma() calls are the only fused operations),
and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libidp.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-fopenmp", "-Wall",
              "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    """Compile every source and link libidp.so; returns the library path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    o = os.path.join(OUT_DIR, "graph.o")
    _run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "graph.cpp"), "-o", o], verbose)
    objs.append(o)
    for src in ("idp_kernels.hip", "idp_adjoint.hip", "idp_capi.hip"):
        o = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
          "-lgomp"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
