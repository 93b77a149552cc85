import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-only test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build()
    return oracle


@pytest.fixture(autouse=True)
def _device_error_word(request):
    """After every GPU test, the library's device error word must be clear."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    import paper_2305_05245_amd as pss

    assert pss.device_check(0) == 0, "a kernel reported a broken invariant"
