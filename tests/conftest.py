import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def box16m():
    """The 16M benchmark workload (16,000,000 polydisperse spheres at volume fraction
    0.3), generated once per session for the tests that need it."""
    import workloads
    print("[test] generating the 16M workload", flush=True)
    box = workloads.config(3)
    assert box.n == 16_000_000
    return box
