import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def hb():
    """The GPU binding; fails loudly when the HIP library or the GPU is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test collected without a visible GPU")
    from paper_1803_01291_amd import hb as _hb
    _hb.load()
    return _hb
