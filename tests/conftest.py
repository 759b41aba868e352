import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def load_counts(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            b, c = line.split()
            out.append(int(c))
    return out


def load_lng(name):
    import numpy as np
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            b, v = line.split()
            out.append(float(v))
    return np.array(out)


@pytest.fixture(scope="session")
def golden():
    class G:
        counts = staticmethod(load_counts)
        lng = staticmethod(load_lng)
        dir = GOLDEN
    return G
