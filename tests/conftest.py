import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: CPU test of several minutes (runs with FFBIE_RUN_SLOW=1)")


HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_collection_modifyitems(config, items):
    """Tests marked slow (several CPU minutes) run only with FFBIE_RUN_SLOW=1."""
    if os.environ.get("FFBIE_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow CPU test: set FFBIE_RUN_SLOW=1")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
