"""CPU check of the host tables behind the one-problem-per-wavefront tree
kernel (elimination schedule, path-pair layout): tests/path_layout_check.cpp
builds them for ~300 trees with the library's own header and carries out the
kernel's lane-by-lane elimination with them in FP64, against a dense solve."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2505_03728_amd", "csrc")


def test_path_layout_tables_and_elimination(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path / "path_layout_check")
    cmd = [cxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(HERE, "path_layout_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout[-2000:])
    assert out.returncode == 0, out.stdout[-4000:]
    assert "0 failures" in out.stdout
