import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def load_golden(name):
    """Parse a tests/golden text fixture: 'key: numbers' lines, ';' separates
    matrix rows, '|' separates lists; '#' starts a comment."""
    path = os.path.join(ROOT, "tests", "golden", name)
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line or ":" not in line:
                continue
            key, val = line.split(":", 1)
            val = val.strip()
            if "|" in val:
                out[key.strip()] = [np.array([float(x) for x in part.split()]) for part in val.split("|")]
            elif ";" in val:
                out[key.strip()] = np.array([[float(x) for x in row.split()] for row in val.split(";")])
            else:
                out[key.strip()] = np.array([float(x) for x in val.split()])
    return out


@pytest.fixture
def golden():
    return load_golden
