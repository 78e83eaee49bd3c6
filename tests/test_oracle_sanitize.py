"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

oracle/sanitize_check.cpp drives every path of the oracle's trajectory solver
(dense and CSR right-hand sides, several channels, the learned proposal with an
out-of-range output, segment records, a jump log shorter than the jump count,
the max_steps and step-size underflow failures, the single-step and jump-free
entry points).  It is built here with g++ -fsanitize=address,undefined and any
report aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sanitize_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "sanitize_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-fopenmp", SRC, "-o", str(exe)]
    subprocess.run(cmd, check=True, cwd=os.path.join(ROOT, "oracle"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitize check ok" in r.stdout
