import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test (oracle on a large grid)")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def mol40():
    from paper_2108_01186_amd import synth
    return synth.make_workload("mol40")


@pytest.fixture(scope="session")
def mol40_oracle(oracle, mol40):
    s = mol40
    return oracle.sic_spin(s.psi[0], s.fod[0], s.n, s.h, s.origin)
