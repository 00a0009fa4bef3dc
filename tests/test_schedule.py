"""CPU check of the persistent work queue the tiled kernels use: the
queue arithmetic of sched.hpp is compiled for the host and exhausted over
many launch shapes (tests/native/sched_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_queue_hands_out_every_item_once(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "sched_check"
    src = os.path.join(ROOT, "tests", "native", "sched_check.cpp")
    inc = ["-I", os.path.join(ROOT, "paper_2309_15595_amd", "csrc"), "-I", os.path.join(ROOT, "include")]
    subprocess.run([hipcc, "-O1", "-std=c++17", *inc, src, "-o", str(exe)], check=True,
                   capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert " 0 violations" in out.stdout
