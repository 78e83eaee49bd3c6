"""Builds the CPU oracle library ``oracle/liboracle.so`` (test infrastructure).

Plain g++ with OpenMP; portable x86-64-v2 code and no floating-point
contraction, so every operation rounds exactly as written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qtm_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-march=x86-64-v2", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
