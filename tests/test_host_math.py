"""Row-split Legendre work lists (host logic, CPU): part coverage and partial
slots, the per-compute-unit balanced dispatch permutation, and the recurrence
checkpoints against the normalised Legendre table."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_18389_amd", "csrc")


def test_work_lists_and_checkpoints(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "host_math_check"
    subprocess.run([cxx, "-O2", "-std=c++17", "-pthread", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "host_math_check.cpp"),
                    os.path.join(CSRC, "host_math.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
