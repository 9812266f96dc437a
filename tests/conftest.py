import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def params():
    import oracle

    return oracle.sm_params()


_ORACLE_CACHE = {}


@pytest.fixture(scope="session")
def oracle_points():
    """(momenta, oracle |M|^2) of the first n seeded RAMBO points of a
    workload, computed once per session (the oracle runs multi-threaded)."""
    import oracle
    from inputs import process_points

    def get(proc, n, seed):
        key = (proc, n, seed)
        if key not in _ORACLE_CACHE:
            mom = process_points(proc, n, seed)
            _ORACLE_CACHE[key] = (mom, oracle.me2(proc, mom))
        return _ORACLE_CACHE[key]

    return get
