import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: oracle cases that take more than a few seconds")


@pytest.fixture(scope="session")
def lib():
    """The HIP library through its Python binding; skips without a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2502_02395_amd import h2
    return h2
