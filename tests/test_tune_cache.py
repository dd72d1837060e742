"""The on-disk tuning cache (CPU): keys, round trip, other entries kept."""
import json

import numpy as np

import graphgen as gg
from paper_2208_04514_amd import tune_cache as T


def test_signature_depends_on_the_csr():
    g, _ = gg.load_config("uniform4096")
    a = T.graph_signature(g.row_ptr, g.col)
    assert a == T.graph_signature(g.row_ptr.copy(), g.col.copy())
    col = g.col.copy()
    col[0] = (col[0] + 1) % g.n
    assert a != T.graph_signature(g.row_ptr, col)
    assert len(a) == 16


def test_round_trip_keeps_other_entries(tmp_path):
    p = str(tmp_path / "t.json")
    assert T.lookup("gfx950", "abc", 1, p) is None
    T.store("gfx950", "abc", 1, {"driver": 3, "alpha": 60.0}, p, note="plain")
    T.store("gfx950", "abc", 4096, {"batch_alpha": 4.0, "batch_big_degree": 128}, p)
    T.store("gfx942", "abc", 1, {"driver": 2}, p)
    assert T.lookup("gfx950", "abc", 1, p) == {"driver": 3, "alpha": 60.0}
    assert T.lookup("gfx950", "abc", 4096, p) == {"batch_alpha": 4.0, "batch_big_degree": 128}
    assert T.lookup("gfx942", "abc", 1, p) == {"driver": 2}
    T.store("gfx950", "abc", 1, {"driver": 4}, p)        # replaces only its own key
    assert T.lookup("gfx950", "abc", 1, p) == {"driver": 4}
    data = json.load(open(p))
    assert set(data) == {"gfx950/abc/1", "gfx950/abc/4096", "gfx942/abc/1"}


def test_unreadable_file_is_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert T.load(str(p)) == {}
    assert T.lookup("gfx950", "x", 1, str(p)) is None
    np.testing.assert_equal(T.load(str(tmp_path / "missing.json")), {})
