"""Builds the CPU oracle libraries (test infrastructure).

``oracle/liboracle.so`` is the parity build: plain g++ with OpenMP, portable
x86-64-v2 code and no floating-point contraction, so every operation rounds
exactly as written in the source.  ``oracle/liboracle_fast.so`` is the same
source built with -O3 for AVX2/FMA hosts (x86-64-v3: the library is built here and
run on a host whose exact CPU model is not known at build time, so it is not tuned
to this machine with -march=native) for timing the oracle as a CPU baseline only
(contraction allowed, so its last bits may differ); no parity check uses it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qtm_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_FAST = os.path.join(HERE, "liboracle_fast.so")
FLAGS = {LIB: ["-O2", "-march=x86-64-v2", "-ffp-contract=off"],
         LIB_FAST: ["-O3", "-march=x86-64-v3"]}


def _build_one(lib: str, verbose: bool) -> str:
    cmd = ["g++", "-std=c++17"] + FLAGS[lib] + ["-fopenmp", "-fPIC", "-shared", "-Wall",
                                               "-Wno-unused-function", SRC, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose: bool = False) -> str:
    _build_one(LIB_FAST, verbose)
    return _build_one(LIB, verbose)


def ensure_built(fast: bool = False) -> str:
    lib = LIB_FAST if fast else LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        _build_one(lib, False)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
