import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950); runs the HIP library")


def load_golden(name):
    """Parses a `key = v v v` fixture under tests/golden/ into lists of ints."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, vals = line.split("=", 1)
            out[key.strip()] = [int(v, 0) for v in vals.split()]
    return out


@pytest.fixture(scope="session")
def golden_example():
    return load_golden("worked_example.txt")
