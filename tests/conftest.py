import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size CPU oracle runs (set FIGARO_SLOW=1)")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("FIGARO_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="full-size oracle run; set FIGARO_SLOW=1")
    for item in items:
        if "slow" in item.keywords and "gpu" not in item.keywords:
            item.add_marker(skip)
