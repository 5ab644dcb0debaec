import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs on the GPU box only)")
    config.addinivalue_line("markers", "slow: long CPU test")


def load_golden(name):
    """Parse a tests/golden/*.txt fixture: '#' comments, then blocks headed by a name."""
    path = os.path.join(ROOT, "tests", "golden", name)
    blocks, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line[0].isalpha() and " " not in line:
                cur = line
                blocks[cur] = []
                continue
            blocks[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


@pytest.fixture(scope="session")
def golden():
    return load_golden
