"""Shared fixtures.  Tests marked ``gpu`` need an MI355X and the built HIP library."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU and the built librmpcast.so")


@pytest.fixture(scope="session")
def tiny_map():
    from paper_2301_08068_amd import workloads as W
    return W.tiny_map(1)


@pytest.fixture(scope="session")
def paper_map():
    from paper_2301_08068_amd import workloads as W
    return W.paper_map(2)


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(12345)
