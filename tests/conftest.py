import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding on cuda:0; GPU tests fail loudly if the library is
    missing (there is no fallback)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU in this container")
    import paper_2104_00792_amd as hg

    hg.lib()  # raises if libhg.so was not built
    torch.cuda.set_device(0)
    return hg
