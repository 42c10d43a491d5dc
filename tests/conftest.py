import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU run (set LBE_SLOW=1 to run)")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("LBE_SLOW"):
        return
    skip = pytest.mark.skip(reason="slow CPU test; set LBE_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
