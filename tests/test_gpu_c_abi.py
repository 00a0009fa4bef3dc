"""The library driven from plain C (tests/native/c_abi_solve.c): a
complex128 and a float64 solve of known-spectrum matrices through the C ABI,
in a child process with no Python or torch in it."""
import subprocess

import pytest

from tests.test_abi import _build_c_example

pytestmark = pytest.mark.gpu


def test_c_program_solves(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    exe = _build_c_example(tmp_path / "c_abi_solve")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert r.stdout.strip().endswith("ok")
