import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_native():
    from oracle import native
    native.build(force=False)
    return native


@pytest.fixture(scope="module")
def ctx():
    """A library context on GPU 0 (GPU tests only)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2603_15023_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch
