import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large inputs; still CPU-only unless also marked gpu")


@pytest.fixture(scope="session")
def dawn():
    """The HIP library binding; skips when no GPU is visible."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_07872_amd as d
    d.load()  # raises if libdawn.so is missing: no silent fallback
    return d
