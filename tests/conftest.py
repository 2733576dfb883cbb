import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its binding; skips cleanly without a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_13612_amd import binding
    return binding.load()


def pytest_collection_modifyitems(config, items):
    """Skip GPU tests when no GPU is visible (CPU container runs -m "not gpu")."""
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
