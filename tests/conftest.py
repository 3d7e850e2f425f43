import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: CPU test of more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _torch_owns_the_device(request):
    """When GPU tests run, initialise torch's device runtime before any test loads
    the library, as a caller does (torch provides the device memory and streams):
    torch and the library then share one HIP runtime from the start, whichever
    test uses torch first."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        try:
            import torch
        except ImportError:
            torch = None
        if torch is not None and torch.cuda.is_available():
            torch.cuda.init()
    yield
