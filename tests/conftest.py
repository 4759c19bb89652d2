import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: runs for minutes (skipped unless LBM_RUN_SLOW=1)")


def pytest_collection_modifyitems(config, items):
    """Tests marked slow (full-length runs against the CPU oracle, several
    minutes of host time each) run only when LBM_RUN_SLOW=1."""
    if os.environ.get("LBM_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="full-length run with minutes of CPU oracle time: set LBM_RUN_SLOW=1 to run it")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def o2lib():
    from oracle import o2
    o2.build(force=False)
    return o2
