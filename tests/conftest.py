"""Shared pytest set-up: markers, import path and the FP64 oracle build."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) device and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU physics run (still part of the CPU suite)")


@pytest.fixture(scope="session", autouse=True)
def _oracle_lib():
    import oracle
    oracle.build(force=False)
    oracle.set_threads(min(8, os.cpu_count() or 1))
    yield
