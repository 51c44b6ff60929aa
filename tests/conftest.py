import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libvie")
    config.addinivalue_line("markers", "slow: long-running CPU oracle check")


@pytest.fixture(scope="session")
def vie_ctx():
    """One libvie context on device 0 for the GPU tests."""
    from paper_2501_13512_amd import vie as V
    ctx = V.vie_context_create(0)
    yield ctx
    V.vie_context_destroy(ctx)
