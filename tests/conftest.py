import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")
    config.addinivalue_line("markers", "long: minutes-long GPU case, run when STOKES_RUN_LONG=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("STOKES_RUN_LONG") == "1":
        return
    skip = pytest.mark.skip(reason="minutes-long 512^3 case; set STOKES_RUN_LONG=1 to run it")
    for item in items:
        if "long" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle
