import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (oracle at larger D)")


def pytest_collection_modifyitems(config, items):
    # deselect slow tests unless asked for explicitly with -m slow
    mexpr = config.getoption("-m") or ""
    if "slow" in mexpr:
        return
    skip = pytest.mark.skip(reason="slow oracle test; run with -m slow")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
