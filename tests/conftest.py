import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def built_library():
    """libgmrf.so, built in-tree if it is not there yet."""
    from paper_1606_00980_amd import build
    if not os.path.exists(build.OUT):
        build.build(verbose=False)
    return build.OUT
