import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def hip():
    """The HIP library binding; GPU tests only."""
    from paper_2311_02101_amd import hp
    lib = hp.load()
    if not hp.device_available():
        pytest.fail("GPU test collected but no HIP device is visible")
    return lib
