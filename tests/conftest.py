import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def rel_err(x, ref):
    """Per-pixel relative error |x - ref| / max(|ref|, 1e-12 max|ref|)."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = 1e-12 * max(float(np.abs(ref).max()), 1e-300)
    return np.abs(x - ref) / np.maximum(np.abs(ref), floor)


@pytest.fixture(scope="session")
def fc():
    """The HIP library binding (built in-tree if nothing is built yet)."""
    import paper_2011_04736_amd as fcat
    if not os.path.exists(fcat.lib_path()):
        from paper_2011_04736_amd import _build
        _build.build()
    fcat.load()
    return fcat
