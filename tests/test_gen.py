"""Generator checks: determinism, CSR validity and the stated shapes of each workload."""
import numpy as np
import pytest

import graphgen as gg


def _valid_csr(g):
    rp, col = g.row_ptr, g.col
    assert rp.dtype == np.int32 and col.dtype == np.int32
    assert rp.shape == (g.n + 1,) and rp[0] == 0 and rp[-1] == col.size
    assert (np.diff(rp.astype(np.int64)) >= 0).all()
    assert ((col >= 0) & (col < g.n)).all()


def _edge_keys(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr.astype(np.int64)))
    return src, g.col.astype(np.int64)


def _simple(g):
    s, d = _edge_keys(g)
    assert (s != d).all(), "self-loop survived"
    key = s * g.n + d
    assert np.unique(key).size == key.size, "repeated edge survived"


def _symmetric(g):
    s, d = _edge_keys(g)
    fwd = np.sort(s * g.n + d)
    rev = np.sort(d * g.n + s)
    assert np.array_equal(fwd, rev)


def test_uniform_exact_m_and_deterministic():
    a = gg.gen_uniform(4096, 32768, 1)
    b = gg.gen_uniform(4096, 32768, 1)
    c = gg.gen_uniform(4096, 32768, 2)
    _valid_csr(a)
    _simple(a)
    assert a.m == 32768
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert not np.array_equal(a.col, c.col)


@pytest.mark.parametrize("scale", [8, 10, 12])
def test_rmat_shape(scale):
    g = gg.gen_rmat(scale, 16, 11)
    _valid_csr(g)
    _simple(g)
    _symmetric(g)
    assert g.n == 1 << scale
    # symmetrised from 16 * n draws, after dedupe: at most 32 * n directed edges
    assert 0 < g.m <= 32 * g.n
    h = gg.gen_rmat(scale, 16, 11)
    assert np.array_equal(g.col, h.col)


def test_rmat_skew():
    g = gg.gen_rmat(12, 16, 3)
    deg = g.out_degree()
    # scale-free: the largest degree is far above the mean
    assert deg.max() > 20 * deg.mean()


def test_grid_counts_and_manhattan_structure():
    k = 16
    g = gg.gen_grid(k, 1, delete_frac=0.0, shortcut_frac=0.0)
    _valid_csr(g)
    _simple(g)
    _symmetric(g)
    assert g.m == 2 * (2 * k * (k - 1))      # 2k(k-1) undirected edges, both directions
    s, d = _edge_keys(g)
    dr = np.abs(s // k - d // k)
    dc = np.abs(s % k - d % k)
    assert ((dr + dc) == 1).all()


def test_grid_damage_and_shortcuts():
    k = 64
    E = 2 * k * (k - 1)
    g = gg.gen_grid(k, 5, delete_frac=0.05, shortcut_frac=0.001)
    _valid_csr(g)
    _simple(g)
    _symmetric(g)
    assert g.meta["deleted"] == int(np.floor(0.05 * E))
    assert g.meta["shortcuts"] == int(np.floor(0.001 * E))
    lo = 2 * (E - g.meta["deleted"])
    assert lo <= g.m <= lo + 2 * g.meta["shortcuts"]


def test_sources_distinct_and_seeded():
    pool = np.arange(100, 200, dtype=np.int32)
    a = gg.sample_sources(pool, 50, 7)
    b = gg.sample_sources(pool, 50, 7)
    assert np.array_equal(a, b)
    assert np.unique(a).size == 50 and np.isin(a, pool).all()


def test_largest_wcc_tie_break():
    # two components of size 3: {0,1,2} and {3,4,5}; the one with node 0 wins
    g = gg.gen_edges(7, [(1, 0), (1, 2), (4, 3), (5, 4)])
    assert gg.largest_wcc_nodes(g).tolist() == [0, 1, 2]


def test_config_small_workloads():
    g, src = gg.load_config("uniform4096", use_cache=False)
    assert g.n == 4096 and g.m == 32768 and src.size == 8
    g, src = gg.load_config("rmat12", use_cache=False)
    wcc = g.meta["wcc_nodes"]
    assert np.isin(src, wcc).all() and src.size == 64


def test_islands_components():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    g = gg.gen_islands(40, 4, 300, 6, seed=3)
    a = csr_matrix((np.ones(g.m, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    nc, lab = connected_components(a, directed=False)
    assert nc == 40
    sizes = np.bincount(lab)
    assert sizes.min() >= 4 and sizes.max() <= 300
    # symmetric, loop-free
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert not (src == g.col).any()
    fwd = set(zip(src.tolist(), g.col.tolist()))
    assert all((v, u) in fwd for u, v in fwd)


def test_weights_seeded_in_range_and_symmetric():
    g, _ = gg.load_config("grid128")
    w = gg.gen_weights(g, 3, 9, seed=5)
    assert w.dtype == np.int32 and w.shape == (g.m,)
    assert w.min() >= 3 and w.max() <= 9
    assert np.array_equal(w, gg.gen_weights(g, 3, 9, seed=5))
    ws = gg.gen_weights(g, 1, 1000, seed=6, symmetric=True)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    fwd = {(int(a), int(b)): int(x) for a, b, x in zip(src, g.col, ws)}
    assert all(fwd[(b, a)] == x for (a, b), x in fwd.items())
    assert len(np.unique(ws)) > 500
