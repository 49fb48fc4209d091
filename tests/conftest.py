import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def load_golden(name):
    """Parse a ``key = value`` fixture; values become floats or lists of floats."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            parts = [float(x) for x in v.split()]
            out[k] = parts[0] if len(parts) == 1 else parts
    return out


@pytest.fixture
def golden():
    return load_golden


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(12345)
