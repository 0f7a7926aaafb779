"""Host check of the multiply-shift division the kernels use to unravel
Khatri-Rao row indices (csrc/cpg_fastdiv.h): compiled with g++ and compared
with the hardware divide by brute force."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fast_division_matches_hardware_divide(tmp_path):
    exe = tmp_path / "fastdiv_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1204_1586_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "fastdiv_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
