import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    # the library is built ahead of time; build it here only if nothing is built
    if not os.path.exists(os.path.join(ROOT, "paper_2503_18616_amd", "libxpbd.so")):
        from paper_2503_18616_amd import build
        build.build()


def f32(v):
    """A parameter as the GPU library sees it: rounded to float32, held in double."""
    return float(np.float32(v))


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
