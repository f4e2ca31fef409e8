import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def oracle():
    import oracle as O

    O.lib()
    return O


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0 (loading fails loudly if it is not built)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07028_amd as P

    P.lib()
    return P
