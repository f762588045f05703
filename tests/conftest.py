import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (oracle at larger sizes)")


def rel_fro(X, Ref):
    """Relative Frobenius error ||X - Ref||_F / ||Ref||_F (absolute when Ref = 0)."""
    import numpy as np
    dt = np.complex128 if (np.iscomplexobj(X) or np.iscomplexobj(Ref)) else np.float64
    X = np.asarray(X, dtype=dt)
    Ref = np.asarray(Ref, dtype=dt)
    d = float(np.linalg.norm(X - Ref))
    r = float(np.linalg.norm(Ref))
    return d / r if r > 0 else d


@pytest.fixture
def relerr():
    return rel_fro
