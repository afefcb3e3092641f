"""Builds libtopktri.so (all HIP sources in csrc/) for gfx950 with hipcc, and the CPU program of
the paper's own exact method, libtopktri_dhl.so (csrc/dhl.cpp, g++), in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtopktri.so")
DHL_LIB = os.path.join(HERE, "libtopktri_dhl.so")
SOURCES = ["graph.hip", "query.hip", "scan.hip", "batch.hip", "approx.hip", "sampling.hip", "cliques.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # strict IEEE evaluation of the FP64 scores: no contraction into FMA
    "-ffp-contract=off",
    # never emit packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build_dhl(force: bool = True) -> str:
    if not force and os.path.exists(DHL_LIB):
        return DHL_LIB
    tmp = DHL_LIB + ".tmp"
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-ffp-contract=off",
                           "-o", tmp, os.path.join(CSRC, "dhl.cpp")])
    os.replace(tmp, DHL_LIB)
    return DHL_LIB


def build(force: bool = True, verbose: bool = False) -> str:
    build_dhl(force)
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
