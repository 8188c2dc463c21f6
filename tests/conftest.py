import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    # the oracle's 2-D transforms split their lines over threads; results do
    # not depend on the count (at most the 16 host cores of one GPU's share)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    return oracle
