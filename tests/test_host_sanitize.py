"""The library's host-side routines (coarsest-level inverses, small inverses, Chebyshev coefficients, the
Faddeev-LeVerrier patch polynomials, the FGMRES least-squares update, the binomial checkpointing schedule) built
on the CPU with the address and undefined-behaviour sanitizers and checked against properties that fix their
results (tests/host_math_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2403_08084_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_math_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_math_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(HERE, "host_math_check.cpp"),
           os.path.join(CSRC, "host_math.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host_math checks passed" in r.stdout
