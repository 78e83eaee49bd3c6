"""Builds libqtm.so (HIP, gfx950) in-tree: paper_1810_03047_amd/libqtm.so.

    python -m paper_1810_03047_amd.build [--jobs N]

Every HIP source is compiled with hipcc for gfx950 with packed FP32
instructions disabled; the objects are linked into one shared library that
exports the C ABI of include/qtm.h.
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqtm.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"
# team-kernel shapes (row tiles per wave x waves per team), one translation unit each
TEAM_SHAPES = ("1x1", "2x1", "1x2", "1x3", "1x4", "2x2", "1x5", "3x2", "5x1", "1x6", "2x3", "1x7", "4x2", "1x8", "2x4", "3x1", "4x1")
EXTRA = ["qtm_wave_batch.hip", "qtm_wave_td0.hip", "qtm_wave_td1.hip", "qtm_expo.hip", "qtm_sparse_r1.hip", "qtm_sparse_r2.hip", "qtm_sparse_r4.hip"]
SOURCES = ["qtm_wave.hip"] + [f"qtm_wave_t{s}.hip" for s in TEAM_SHAPES] + EXTRA + ["qtm_dense.hip", "qtm_sparse.hip",
                                                                     "qtm_mlp.hip", "qtm_capi.cpp"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wno-unused-result"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, src + ".o")
    cmd = ["hipcc"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC"] + objs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.verbose, a.jobs))


if __name__ == "__main__":
    main()
