"""Pins for the CPU oracle, against what the paper and the mathematics fix.

None of these retypes the oracle: each compares it with an independent
algorithm (Floyd–Warshall; Theorem 1's boolean matrix powers; scipy's
unweighted shortest paths), with a closed form, with hand-derived fixtures, or
with invariants that hold at any size.  A plausible slip in the oracle — a LIFO
instead of a FIFO queue, in-edges instead of out-edges, an off-by-one level, a
missing visited check — breaks at least one of them (see the planted-mistake
tests at the bottom, which run on the CPU against the pins' own checkers).
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from conftest import load_golden


# ---------------------------------------------------------------------------
# hand-derived fixtures
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,sym", [("hand_directed10.txt", False), ("petersen.txt", True)])
def test_golden(name, sym):
    n, edges, rows = load_golden(name)
    # keep self-loops and repeats: they must not change distances
    g = gg.gen_edges(n, edges, drop_self=False, dedupe=False)
    for s, want in rows.items():
        assert np.array_equal(oracle.sssp(g, s), want), (name, s)
    if sym:
        # Petersen: distance-regular, diameter 2 -> 1 x 0, 3 x 1, 6 x 2 from every vertex
        for s in range(n):
            assert np.bincount(oracle.sssp(g, s)).tolist() == [1, 3, 6]


# ---------------------------------------------------------------------------
# independent algorithms on tiny graphs
# ---------------------------------------------------------------------------

def _tiny_graphs(count=500, seed=2026):
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(rng.integers(1, 49))
        p = float(rng.choice([0.02, 0.05, 0.1, 0.2, 0.5]))
        m = rng.binomial(n * n, p)
        u = rng.integers(0, n, size=m)
        v = rng.integers(0, n, size=m)
        sym = bool(i % 3 == 0)
        # inject self-loops and repeats: accepted, never change distances
        g = gg.gen_edges(n, np.stack([u, v], 1), symmetrize=sym, drop_self=False,
                         dedupe=bool(i % 2))
        yield i, g


def test_oracle_vs_floyd_warshall_and_theorem1():
    for i, g in _tiny_graphs():
        a = oracle.adjacency(g)
        fw = oracle.floyd_warshall(a)
        # Theorem 1 needs i != j; the diagonal is 0 by definition
        bp = oracle.bool_power_distances(a)
        assert np.array_equal(fw, bp), f"graph {i}: FW vs boolean powers"
        bfs = oracle.mssp(g, np.arange(g.n, dtype=np.int32))
        assert np.array_equal(bfs, fw), f"graph {i}: BFS vs FW"


def test_oracle_vs_scipy_unweighted():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path

    for seed, (n, m) in enumerate([(500, 1500), (2000, 4000), (1500, 30000)]):
        g = gg.gen_uniform(n, m, 40 + seed)
        a = csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(n, n))
        src = gg.sample_sources(n, 20, seed)
        ref = shortest_path(a, directed=True, unweighted=True, indices=src)
        ref = np.where(np.isinf(ref), -1, ref).astype(np.int32)
        assert np.array_equal(oracle.mssp(g, src, threads=4), ref)


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def test_directed_path():
    n = 50
    g = gg.gen_edges(n, [(i, i + 1) for i in range(n - 1)])
    for s in (0, 17, 49):
        v = np.arange(n)
        assert np.array_equal(oracle.sssp(g, s), np.where(v >= s, v - s, -1))


def test_directed_and_undirected_cycle():
    n = 37
    e = [(i, (i + 1) % n) for i in range(n)]
    g = gg.gen_edges(n, e)
    gs = gg.gen_edges(n, e, symmetrize=True)
    v = np.arange(n)
    for s in (0, 5, 36):
        assert np.array_equal(oracle.sssp(g, s), (v - s) % n)
        dd = np.abs(v - s)
        assert np.array_equal(oracle.sssp(gs, s), np.minimum(dd, n - dd))


def test_stars_complete_empty():
    n = 40
    out_star = gg.gen_edges(n, [(0, i) for i in range(1, n)])
    in_star = gg.gen_edges(n, [(i, 0) for i in range(1, n)])
    want = np.ones(n, np.int32)
    want[0] = 0
    assert np.array_equal(oracle.sssp(out_star, 0), want)
    leaf = oracle.sssp(out_star, 3)          # out-degree 0 source: only itself
    assert leaf[3] == 0 and (np.delete(leaf, 3) == -1).all()
    d = oracle.sssp(in_star, 5)
    assert d[5] == 0 and d[0] == 1 and (np.delete(d, [0, 5]) == -1).all()
    assert (oracle.sssp(in_star, 0)[1:] == -1).all()
    comp = gg.gen_edges(n, [(i, j) for i in range(n) for j in range(n) if i != j])
    for s in (0, 13):
        d = oracle.sssp(comp, s)
        assert d[s] == 0 and (np.delete(d, s) == 1).all()
    empty = gg.gen_edges(n, np.zeros((0, 2), np.int64))
    d = oracle.sssp(empty, 7)
    assert d[7] == 0 and (np.delete(d, 7) == -1).all()


def test_grid_manhattan():
    k = 45
    g = gg.gen_grid(k, 0, delete_frac=0.0, shortcut_frac=0.0)
    r, c = np.divmod(np.arange(k * k), k)
    for s in (0, 17 * k + 3, k * k - 1):
        sr, sc = divmod(s, k)
        assert np.array_equal(oracle.sssp(g, s), np.abs(r - sr) + np.abs(c - sc))
    # damage without shortcuts can only lengthen paths
    gd = gg.gen_grid(k, 4, delete_frac=0.05, shortcut_frac=0.0)
    for s in (0, 1000):
        sr, sc = divmod(s, k)
        d = oracle.sssp(gd, s)
        man = np.abs(r - sr) + np.abs(c - sc)
        assert ((d == -1) | (d >= man)).all()


def test_hypercube_hamming():
    dim = 9
    n = 1 << dim
    e = [(v, v ^ (1 << b)) for v in range(n) for b in range(dim)]
    g = gg.gen_edges(n, e)
    pop = np.array([bin(x).count("1") for x in range(n)])
    for s in (0, 77, n - 1):
        assert np.array_equal(oracle.sssp(g, s), pop[np.arange(n) ^ s])


# ---------------------------------------------------------------------------
# invariants at workload size
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["uniform4096", "rmat12", "grid128", "grid128ns"])
def test_invariants_on_workloads(name):
    g, src = gg.load_config(name)
    for s in src[:8]:
        d = oracle.sssp(g, int(s))
        oracle.check_invariants(g, int(s), d)


def test_mssp_rows_threads_duplicates():
    g, src = gg.load_config("rmat12")
    srcs = np.concatenate([src[:10], src[:3]]).astype(np.int32)
    one = np.stack([oracle.sssp(g, int(s)) for s in srcs])
    for t in (1, 3, 8):
        assert np.array_equal(oracle.mssp(g, srcs, threads=t), one)
    assert oracle.mssp(g, np.empty(0, np.int32)).shape == (0, g.n)
    # permuting the sources permutes the rows
    p = np.random.default_rng(0).permutation(srcs.size)
    assert np.array_equal(oracle.mssp(g, srcs[p], threads=2), one[p])


def test_bad_arguments_rejected():
    g = gg.gen_edges(4, [(0, 1)])
    with pytest.raises(ValueError):
        oracle.sssp(g, 4)
    with pytest.raises(ValueError):
        oracle.mssp(g, np.array([0, -1], np.int32))


# ---------------------------------------------------------------------------
# largest WCC
# ---------------------------------------------------------------------------

def test_wcc_vs_scipy():
    for name in ("uniform4096", "rmat12", "rmat14", "grid128"):
        g, _ = gg.load_config(name)
        assert np.array_equal(oracle.largest_wcc(g), gg.largest_wcc_nodes(g)), name
    rng = np.random.default_rng(5)
    for i in range(60):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(0, 2 * n))
        e = rng.integers(0, n, size=(m, 2))
        g = gg.gen_edges(n, e)
        assert np.array_equal(oracle.largest_wcc(g), gg.largest_wcc_nodes(g)), i


def test_wcc_directed_tie_break():
    # {0,1} via 1->0, and {2,3} via 2->3: equal sizes, the one holding 0 wins
    g = gg.gen_edges(5, [(1, 0), (2, 3)])
    assert oracle.largest_wcc(g).tolist() == [0, 1]
    g = gg.gen_edges(5, [(4, 3), (2, 3), (0, 1)])
    assert oracle.largest_wcc(g).tolist() == [2, 3, 4]


# ---------------------------------------------------------------------------
# the pins catch planted mistakes (mistakes planted in a Python copy on the CPU)
# ---------------------------------------------------------------------------

def _bfs_variant(g, s, mistake):
    """Python BFS with one deliberate slip; used only to show the pins bite."""
    from collections import deque
    rp, col = g.row_ptr, g.col
    if mistake == "in_edges":                 # transposed operand
        src = np.repeat(np.arange(g.n), np.diff(rp))
        order = np.argsort(col, kind="stable")
        rp = np.concatenate([[0], np.cumsum(np.bincount(col, minlength=g.n))])
        col = src[order]
    # "zero_sentinel": the paper's literal 0 = unvisited, which lets an edge
    # back into s overwrite dist[s]
    unvisited = 0 if mistake == "zero_sentinel" else -1
    dist = np.full(g.n, unvisited, np.int64)
    dist[s] = 0
    q = deque([s])
    while q:
        u = q.pop() if mistake == "lifo" else q.popleft()
        for v in col[rp[u]:rp[u + 1]]:
            if dist[v] == unvisited:
                dist[v] = dist[u] + (2 if mistake == "step2" else 1)
                q.append(int(v))
    if mistake == "zero_sentinel":
        dist = np.where((dist == 0) & (np.arange(g.n) != s), -1, dist)
    return dist.astype(np.int32)


@pytest.mark.parametrize("mistake", ["lifo", "in_edges", "step2", "zero_sentinel"])
def test_pins_detect_planted_mistakes(mistake):
    caught = False
    for i, g in _tiny_graphs(count=60, seed=99):
        if g.n < 4:
            continue
        fw = oracle.floyd_warshall(oracle.adjacency(g))
        bad = np.stack([_bfs_variant(g, s, mistake) for s in range(g.n)])
        if not np.array_equal(bad, fw):
            caught = True
            break
    assert caught, f"planted mistake {mistake!r} was not caught by Floyd–Warshall"
    # the correct variant passes the same check
    for i, g in _tiny_graphs(count=20, seed=99):
        fw = oracle.floyd_warshall(oracle.adjacency(g))
        good = np.stack([_bfs_variant(g, s, "none") for s in range(g.n)])
        assert np.array_equal(good, fw)


def test_invariant_checker_detects_corruption():
    g, src = gg.load_config("rmat12")
    s = int(src[0])
    d = oracle.sssp(g, s)
    oracle.check_invariants(g, s, d)
    reached = np.nonzero(d > 1)[0]
    one_deeper = d.copy()
    one_deeper[reached[0]] += 1                 # a node one level too deep
    dropped = d.copy()
    dropped[reached[1]] = -1                    # a reached node reported unreachable
    shortcut = d.copy()
    shortcut[reached[2]] = 1                    # a level-2+ node claimed at level 1
    for bad in (one_deeper, dropped, shortcut):
        with pytest.raises(AssertionError):
            oracle.check_invariants(g, s, bad.astype(np.int32))
