"""CPU checks of the persistent work queue and split-K planner the tiled
kernels use: the queue arithmetic of sched.hpp and the planner of
schedule.cpp are compiled for the host and exhausted over many launch shapes
(tests/native/sched_check.cpp, tests/native/plan_check.cpp); a second build
of each runs under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only: every -fsanitize= follows -Xarch_host)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_15595_amd", "csrc")
SANITIZE = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


def _hipcc():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    return hipcc


def _build_and_run(tmp_path, name, sources, extra):
    exe = tmp_path / name
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    subprocess.run([_hipcc(), "-O1", "-std=c++17", *extra, *inc, *sources, "-o", str(exe)], check=True,
                   capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert " 0 violations" in out.stdout
    return out.stdout


@pytest.mark.parametrize("sanitized", [False, True], ids=["plain", "asan-ubsan"])
def test_queue_hands_out_every_item_once(tmp_path, sanitized):
    _build_and_run(tmp_path, "sched_check", [os.path.join(ROOT, "tests", "native", "sched_check.cpp")],
                   SANITIZE if sanitized else [])


@pytest.mark.parametrize("sanitized", [False, True], ids=["plain", "asan-ubsan"])
def test_planner_keeps_to_its_caps_and_covers_k(tmp_path, sanitized):
    out = _build_and_run(tmp_path, "plan_check",
                         [os.path.join(ROOT, "tests", "native", "plan_check.cpp"), os.path.join(CSRC, "schedule.cpp")],
                         SANITIZE if sanitized else [])
    assert "split along K" in out and not out.startswith("0 plans")
