"""Host code under the address and undefined-behaviour sanitizers: the
assembly planner (csrc/plan.cpp: validation, 1-D tables, the interpolation
set-ups of the three surrogate variants, the tile lists with their row
coverage) and the oracle's C part (every entry point, all maps and
coefficient kinds).  Built with gcc/g++ from the sources; CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined"]
ENV = dict(os.environ, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", ASAN_OPTIONS="detect_leaks=0",
           OMP_NUM_THREADS="2")


def _run(cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout and "runtime error" not in r.stderr, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_c_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", *SAN, "-fopenmp", os.path.join(ROOT, "oracle", "igs_oracle.c"),
          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe], exe)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="no g++ or HIP headers")
def test_planner_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_san")
    csrc = os.path.join(ROOT, "paper_1904_06971_amd", "csrc")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
          "-I" + os.path.join(ROOT, "include"), "-I" + csrc, os.path.join(csrc, "plan.cpp"),
          os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"), "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe], exe)
