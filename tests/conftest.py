import os
import sys

import pytest

# GPU tests run the query server in its layout for 8 or more hardware queues
# (one stage per tier, six lanes); a test switches to the four-queue layout by
# setting the variable lower before it creates a server.  HIP reads the
# variable once, when its runtime starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 12:
    os.environ["GPU_MAX_HW_QUEUES"] = "12"

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle
