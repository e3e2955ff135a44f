import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def load_golden(name):
    """Parse a tests/golden matrix file into {name: 2-D list of floats}."""
    out, cur = {}, None
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                out[cur] = []
            else:
                out[cur].append([float(t) for t in line.split()])
    return out


@pytest.fixture(scope="session")
def golden():
    return load_golden
