import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C ABI)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs (set GRMHD_SLOW=1)")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("GRMHD_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow oracle run; set GRMHD_SLOW=1")
    for it in items:
        if it.get_closest_marker("slow") is not None:
            it.add_marker(skip)
