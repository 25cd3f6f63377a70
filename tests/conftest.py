import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running (large grids)")


@pytest.fixture(scope="session")
def rve_inputs():
    """Seeded workload arrays, generated once per session (the 512^3 sphere
    packings take tens of seconds each): ``rve_inputs(name)`` -> (kappa, info)."""
    import rvegen

    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = rvegen.make_config(name)
        return cache[name]

    return get
