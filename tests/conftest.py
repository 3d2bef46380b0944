import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def cr():
    """The C-ABI binding.  A tree without a built library builds it first (hipcc cross-compiles for
    gfx950 without a GPU); loading then fails loudly if the build did not produce it."""
    from paper_1608_02227_amd import build as _build
    from paper_1608_02227_amd import cr as _cr
    if not os.path.exists(_build.LIB):
        _build.build()
    _cr.load()
    return _cr
