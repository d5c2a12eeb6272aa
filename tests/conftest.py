import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: large CPU oracle case (minutes)")


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def native_lib():
    """The built HIP library (built once here if nothing is built yet)."""
    from paper_1008_2410_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1008_2410_amd import build
        build.build_library()
    return _lib.load()


@pytest.fixture(scope="session")
def fmm_mod(native_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1008_2410_amd import fmm
    return fmm
