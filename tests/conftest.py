import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")
    config.addinivalue_line("markers", "long_measurement: GPU measurement of several minutes; runs only "
                                       "with REWL_LONG_MEASUREMENTS=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("REWL_LONG_MEASUREMENTS") == "1":
        return
    skip = pytest.mark.skip(reason="long measurement (minutes); set REWL_LONG_MEASUREMENTS=1 to run it")
    for item in items:
        if "long_measurement" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    from oracle.build import build_oracle
    build_oracle()
    return oracle
