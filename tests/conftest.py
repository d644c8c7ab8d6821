import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_collection_modifyitems(config, items):
    # GPU tests fail loudly (not skip) when the GPU or the library is missing:
    # selecting them with -m gpu on a machine without a GPU is an error.
    pass


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not oracle.LIB_PATH.exists():
        oracle.build()
    return oracle
