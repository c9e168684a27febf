import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built C-ABI library on a visible GPU; skips when either is absent
    only for tests that are not marked gpu (gpu tests fail loudly instead)."""
    import paper_2305_20053_amd as saa
    saa.require_gpu()
    return saa
