import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU case")


@pytest.fixture(scope="session")
def parity_problem():
    import synth
    return synth.make_problem(**synth.CFG_PARITY)


@pytest.fixture(scope="session")
def parity_oracle(parity_problem):
    import oracle
    p = parity_problem
    return oracle.chase(p.A, oracle.Params(nev=p.nev, nex=p.nex, deg=p.deg, tol=p.tol),
                        V0=p.V0, starts=p.starts)


@pytest.fixture(autouse=True, scope="module")
def _release_device_cache():
    """Give torch's cached device blocks back after every test module, so the
    process holds little device memory when it exits (the next process on the
    GPU starts while the driver is still reclaiming what this one freed)."""
    yield
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    except Exception:
        pass
