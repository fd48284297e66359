import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU run (still minutes at most)")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.set_threads(int(os.environ.get("ORACLE_THREADS", "0")) or (os.cpu_count() or 1))
    return O
