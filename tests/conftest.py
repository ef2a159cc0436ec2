import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    import oracle as _oracle
    _oracle._load()
    return _oracle


@pytest.fixture(scope="session")
def native():
    """libapsp.so loaded through ctypes (built in-tree first if missing)."""
    from paper_2310_03983_amd import build as _build
    import os as _os
    if not _os.path.exists(_build.LIB):
        _build.build()
    from paper_2310_03983_amd import apsp as _apsp
    return _apsp


@pytest.fixture(scope="session")
def dev():
    """The GPU the parity tests run on; fails (does not skip) without one."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    return torch.device("cuda:0")
