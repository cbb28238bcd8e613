import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: oracle runs of tens of seconds")


@pytest.fixture(scope="session")
def torch_cuda():
    """torch with its HIP runtime initialised.  torch's lazy initialisation
    reports no GPU when it first runs after the library has already
    initialised HIP in the process, so a GPU session starts it before any
    test (see pytest_collection_modifyitems) and tests that hand torch
    memory to the library take it from here."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("torch sees no GPU")
    return torch


def pytest_collection_modifyitems(config, items):
    if any(it.get_closest_marker("gpu") for it in items):
        try:
            import torch
            torch.cuda.is_available()   # initialise before the library does
        except Exception:
            pass
