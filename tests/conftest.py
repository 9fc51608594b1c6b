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
def gpu_lib():
    """The HIP library through its C ABI; skips when no GPU is visible."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2106_10913_amd import awg
    return awg


@pytest.fixture(autouse=True, scope="module")
def _release_device_memory():
    """After each module that used the GPU: return the library's cached device
    blocks and torch's cached blocks to the driver, so one module's large
    set-ups do not crowd the device for the next."""
    yield
    awg = sys.modules.get("paper_2106_10913_amd.awg")
    torch = sys.modules.get("torch")
    if awg is None or torch is None or not torch.cuda.is_initialized():
        return
    torch.cuda.synchronize()
    awg.free_cached_memory()
    torch.cuda.empty_cache()
