import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def read_table(name):
    """Parse a golden shell table: returns r and rows (k, a, b, w)."""
    r, rows = None, []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "r":
                r = float(parts[1])
            else:
                rows.append((int(parts[0]), int(parts[1]), int(parts[2]), float(parts[3])))
    return r, rows


@pytest.fixture(scope="session", autouse=True)
def _oracle_threads():
    """The oracle runs on small grids in the tests: one thread avoids OpenMP
    synchronisation costs that dominate at these sizes."""
    import oracle
    prev = oracle.set_threads(0)
    oracle.set_threads(1)
    yield
    oracle.set_threads(prev)
