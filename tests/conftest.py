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


@pytest.fixture(autouse=True)
def _progress_to_terminal(request):
    """Progress lines of the GPU tests (helpers.progress) go to the terminal
    with pytest's output capture suspended, so that they appear under -q too."""
    import helpers
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def write(msg):
        if capman is None:
            print(msg, flush=True)
            return
        capman.suspend_global_capture(in_=False)
        try:
            print(msg, flush=True)
        finally:
            capman.resume_global_capture()

    helpers.set_progress_writer(write)
    yield
    helpers.set_progress_writer(None)
