"""Shared fixtures.  Tests marked `gpu` need an MI355X and the built libimm.so; every other
test runs on the CPU (oracle pins, host logic, library load and symbol checks)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built libimm.so")
    config.addinivalue_line("markers", "slow: full-size workload (minutes on the CPU oracle)")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def imm_gpu():
    """The GPU binding, initialised on device 0 (fails loudly if the library is missing)."""
    import paper_2009_07325_amd as imm
    imm.lib()
    imm.imm_init(0)
    return imm
