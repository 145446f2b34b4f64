import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """The parity totals of the run: how many trees were compared and every
    near tie that was excused, with its margin."""
    from tests import parity
    text = parity.summary()
    if text:
        terminalreporter.write_line(text)
