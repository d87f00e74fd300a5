import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The host-sanitizer test reruns the oracle's tests against an instrumented build of the
# oracle library named here (the default build is used otherwise).
if os.environ.get("WK_ORACLE_LIB"):
    import oracle
    oracle._LIB = os.environ["WK_ORACLE_LIB"]


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
