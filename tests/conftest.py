"""Test configuration: the ``gpu`` marker and shared seeded inputs."""
import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs")


@functools.lru_cache(maxsize=None)
def inputs(cid, pairs=None):
    """Rendered inputs of a configuration, cached per test session."""
    from synth import scene
    return scene.make_inputs(cid, pairs)


@pytest.fixture(scope="session")
def c1_inputs():
    return inputs("c1")


@pytest.fixture(scope="session")
def c2_inputs():
    return inputs("c2")
