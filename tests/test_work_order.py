"""Host test of the XCD-aware launch order of the batched and served launches: a C++ program built with
g++ against the header that holds it (no GPU, no HIP)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_xcd_grouped_order(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = tmp_path / "work_order_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_2302_12454_amd", "csrc"),
                    os.path.join(ROOT, "tests", "work_order_check.cpp"), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout + res.stderr
