import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large inputs")


def pytest_collection_modifyitems(config, items):
    # Full-size GPU tests run late so cheap failures surface first; the
    # allocation-free entry point's tests run last of all.
    def rank(it):
        if "test_zz_no_alloc" in it.nodeid:
            return 2
        return 1 if it.get_closest_marker("gpu") and "full" in it.name else 0
    items.sort(key=rank)
