"""Host-side AddressSanitizer + UndefinedBehaviorSanitizer runs of the CPU code:
the FP64 oracle with the input generators, and the row planner the GPU
library uses (plain C / C++, no GPU).  Each driver exercises every entry
point on small seeded inputs; a sanitizer report or a failed check ends the
driver with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
       "-O1"]


def _run(cmd, tmp_path, exe, env_extra=None):
    out = os.path.join(tmp_path, exe)
    r = subprocess.run(cmd + ["-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([out], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    cmd = ["gcc", "-std=gnu11", "-fopenmp", *SAN,
           os.path.join(ROOT, "tests", "sanitize", "drive_oracle.c"),
           os.path.join(ROOT, "oracle", "tf_oracle.c"), os.path.join(ROOT, "synth", "synth.c"), "-lm"]
    assert "ok" in _run(cmd, str(tmp_path), "drive_oracle")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_row_planner_under_asan_ubsan(tmp_path):
    cmd = ["g++", "-std=c++17", *SAN, os.path.join(ROOT, "tests", "sanitize", "drive_plan.cpp"),
           os.path.join(ROOT, "paper_1410_5209_amd", "csrc", "plan.cpp")]
    assert "ok" in _run(cmd, str(tmp_path), "drive_plan")
