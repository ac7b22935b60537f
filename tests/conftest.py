"""Shared test set-up: the `gpu` marker and on-demand builds of the oracle."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI of libgray)")


@pytest.fixture(scope="session")
def orc():
    """The FP64 CPU oracle, built on first use if no build exists."""
    import oracle
    if not os.path.exists(oracle._LIB):
        oracle.build()
    oracle.lib()
    return oracle
