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


@pytest.fixture(scope="session")
def ct24_reference():
    """The small non-negative CT problem (24^2, 18 angles, 35 bins, alpha 0.05)
    and its minimiser by 100000 iterations of the diagonally preconditioned
    explicit PDHG, shared by the oracle's CT convergence pins."""
    import oracle as O
    import synth
    u, eta = synth.phantom_and_noise(24, 24, 5, 5, (18, 35))
    A = O.joseph(24, 24, synth.parallel_beam_angles(18), 35, 2.0 / 24, 2.0 / 24)
    Au = A.apply(u)
    b = Au + 0.01 * Au.max() * eta
    alpha = 0.05
    return A, b, alpha, O.pdhg_explicit(A, b, alpha, 1, 100000)
