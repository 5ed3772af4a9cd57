import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build
    srcs = [os.path.join(build.HERE, f) for f in ("oracle.cpp", "oracle3.cpp", "oracle.h")]
    if not os.path.exists(build.LIB) or os.path.getmtime(build.LIB) < max(os.path.getmtime(f) for f in srcs):
        build.build()
