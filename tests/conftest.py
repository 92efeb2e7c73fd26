import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def rel_err(x, ref):
    """Normwise error max|x - ref| / max|ref| (the tolerance measure)."""
    import numpy as np
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = float(np.max(np.abs(ref)))
    if den == 0.0:
        return float(np.max(np.abs(x)))
    return float(np.max(np.abs(x - ref))) / den
