import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU runs (still minutes at most)")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import build_oracle, oracle
    if not os.path.exists(oracle.LIB_PATH):
        build_oracle.build()
    return oracle
