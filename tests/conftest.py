import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def lib():
    """The HIP library binding; skips on machines without a GPU."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0812_amd as rb

    return rb
