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
