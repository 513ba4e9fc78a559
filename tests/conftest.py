import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the device)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def pytest_report_header(config):
    return "sst: oracle pins run on CPU; -m gpu parity tests need the built library and a GPU"
