import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~20 s")


@pytest.fixture(scope="session")
def orc():
    import oracle
    for name in ("liborc64.so", "liborc80.so"):
        if not os.path.exists(os.path.join(ROOT, "oracle", name)):
            from oracle import build
            build.build()
            break
    return oracle
