import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The library fills every floating-point device block it hands out with NaN
# bit patterns, so a kernel that reads memory nobody wrote fails its test
# instead of passing on whatever a fresh or recycled block happened to hold.
os.environ.setdefault("FMDDM_POISON_ALLOC", "1")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")
