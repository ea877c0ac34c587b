import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test of several minutes; runs only with "
                                       "GBMC_RUN_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("GBMC_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow CPU pin: set GBMC_RUN_SLOW=1 to run it")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
