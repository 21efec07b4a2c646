import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    # the oracle is plain C; build it if nothing is built yet
    from oracle import oracle as _o
    if not os.path.exists(_o.LIB_PATH):
        _o.build()


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as _o
    return _o
