import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: larger CPU-only oracle checks")


def pytest_collection_modifyitems(config, items):
    # Parity tests need the device; mark-based selection handles the split,
    # this only makes a missing GPU skip (not fail) when -m gpu is not given.
    pass
