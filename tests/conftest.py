import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU-side verification")


def _flush_case(item):
    # Name the case before it touches the GPU, so a fault that ends the
    # process still leaves the case's name in the log.
    if item.get_closest_marker("gpu") is not None:
        sys.stdout.write(f"\n[gpu-case] {item.nodeid}\n")
        sys.stdout.flush()


@pytest.hookimpl(tryfirst=True)
def pytest_runtest_setup(item):
    _flush_case(item)
