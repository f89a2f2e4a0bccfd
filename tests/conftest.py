import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu():
    """Session fixture for GPU tests: fails (never skips) when no GPU is visible."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    from paper_1301_7530_amd import Context

    ctx = Context(0)
    yield ctx
    ctx.close()
