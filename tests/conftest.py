import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: full-size workloads")


def load_golden(name):
    """Parse a tests/golden fixture: returns (n, edge pairs, {source: expected row})."""
    n, edges, rows = None, [], {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "n":
                n = int(t[1])
            elif t[0] == "e":
                edges.append((int(t[1]), int(t[2])))
            elif t[0] == "d":
                rows[int(t[1])] = np.array([int(x) for x in t[2:]], dtype=np.int32)
    return n, edges, rows
