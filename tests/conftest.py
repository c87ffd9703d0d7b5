import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def ctx():
    """A library context on cuda:0 bound to torch's current stream."""
    import torch
    import paper_2411_00688_amd as T
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    c = T.tvs_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    T.tvs_ctx_destroy(c)
