import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


_CACHE = {}


@pytest.fixture(scope="session")
def workload_cache():
    """Seeded workloads shared across tests (they are deterministic)."""
    import workloads

    def get(key, fn=None):
        if key not in _CACHE:
            if fn is not None:
                _CACHE[key] = fn()
            elif isinstance(key, tuple) and key[0] == "workload":
                _CACHE[key] = workloads.workload(*key[1:])
            else:
                raise KeyError(key)
        return _CACHE[key]

    return get
