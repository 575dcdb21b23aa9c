import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running case")


def _print_case(item):
    # Name the case before it touches the GPU, so a run that ends abruptly
    # still shows which test was running.
    if item.get_closest_marker("gpu") is not None:
        sys.stdout.write(f"\n[case] {item.nodeid}\n")
        sys.stdout.flush()


def pytest_runtest_setup(item):
    _print_case(item)
