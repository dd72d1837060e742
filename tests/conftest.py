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


def header_functions():
    """Names of the functions declared in include/dawn.h."""
    import re
    with open(os.path.join(ROOT, "include", "dawn.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dawn_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="session")
def dawn_lib():
    from paper_2208_04514_amd import dawn as D
    return D.load()


@pytest.fixture(scope="session")
def ctx(dawn_lib):
    """One context on device 0 for the whole GPU session (fails loudly without a GPU)."""
    from paper_2208_04514_amd import dawn as D
    h = D.dawn_create(0, 0)
    yield h
    D.dawn_destroy(h)


_GRAPHS = {}


@pytest.fixture(scope="session")
def upload(ctx):
    """upload(name_or_graph) -> (graph handle, Graph, sources); cached per session."""
    import graphgen as gg
    from paper_2208_04514_amd import dawn as D

    def _up(key):
        if isinstance(key, str):
            if key not in _GRAPHS:
                g, src = gg.load_config(key)
                _GRAPHS[key] = (D.dawn_graph_upload(ctx, g.row_ptr, g.col), g, src)
            return _GRAPHS[key]
        g = key
        return D.dawn_graph_upload(ctx, g.row_ptr, g.col), g, None
    return _up
