import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    return oracle.lib()


def pytest_collection_modifyitems(config, items):
    # GPU tests need the ROCm kernel driver; on a machine without one they are
    # skipped (the CPU suite is selected with -m "not gpu" anyway).
    if os.path.exists("/dev/kfd"):
        return
    skip = pytest.mark.skip(reason="no AMD GPU (/dev/kfd) on this machine")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
