import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


def pytest_collection_modifyitems(config, items):
    # keep GPU tests from running on a machine with no GPU when selected by marker
    pass


@pytest.fixture(scope="session", autouse=True)
def _torch_runtime_first(request):
    """GPU tests hand torch device tensors to the library.  Torch's HIP
    runtime has to come up before the library's first GPU call in the
    process (torch reports no GPUs when it initialises after), so a session
    that runs GPU tests initialises it first, whatever the test order."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        import torch

        if torch.cuda.is_available():
            torch.cuda.init()
    yield
