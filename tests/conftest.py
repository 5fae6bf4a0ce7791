import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: oracle checks that take tens of seconds on the CPU")


def load_golden(name):
    """Parse a text fixture of '[label RxC]' headed integer/float blocks."""
    path = os.path.join(ROOT, "tests", "golden", name)
    blocks, cur, label = {}, None, None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                label = line[1:-1].split()[0]
                cur = []
                blocks[label] = cur
            else:
                cur.append([float(t) for t in line.split()])
    import numpy as np
    return {k: np.array(v) for k, v in blocks.items()}
