"""Pins of the weighted oracle (Dijkstra over non-negative integer weights):
the (min, +) extension the paper names as future work (Section 5), for which
the plain definition is the minimum over paths of the summed weights.

Pinned by an independent algorithm (weighted Floyd–Warshall) on tiny graphs
with zero weights, self-loops and repeated edges; by scipy's Dijkstra (a
library routine) on mid-size graphs; by the unweighted oracle when every
weight is 1; by closed forms; by the invariants of exact distances at
workload size; and planted mistakes must fail the Floyd–Warshall pin."""
import numpy as np
import pytest

import graphgen as gg
import oracle


def _tiny_weighted(count=300, seed=7):
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(rng.integers(1, 41))
        p = float(rng.choice([0.03, 0.08, 0.2, 0.5]))
        m = rng.binomial(n * n, p)
        u = rng.integers(0, n, size=m)
        v = rng.integers(0, n, size=m)
        g = gg.gen_edges(n, np.stack([u, v], 1), symmetrize=bool(i % 3 == 0),
                         drop_self=False, dedupe=bool(i % 2))
        hi = int(rng.choice([1, 3, 20, 1000]))
        w = rng.integers(0, hi + 1, size=g.m).astype(np.int32)   # zeros included
        yield i, g, w


def test_dijkstra_vs_floyd_warshall():
    for i, g, w in _tiny_weighted():
        fw = oracle.floyd_warshall_weighted(g, w)
        dj = oracle.wmssp(g, w, np.arange(g.n, dtype=np.int32), threads=2)
        assert np.array_equal(dj, fw), f"graph {i}: Dijkstra vs Floyd–Warshall"


def test_dijkstra_vs_scipy():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import dijkstra

    for seed, (n, m) in enumerate([(600, 3000), (3000, 12000), (2000, 40000)]):
        g = gg.gen_uniform(n, m, 60 + seed)
        w = gg.gen_weights(g, 1, 50, seed=seed)
        src = np.repeat(np.arange(n), np.diff(g.row_ptr))
        # weights >= 1 (a sparse matrix drops explicit zeros); edges are unique
        a = coo_matrix((w.astype(np.float64), (src, g.col)), shape=(n, n)).tocsr()
        s = gg.sample_sources(n, 16, seed)
        ref = dijkstra(a, directed=True, indices=s)
        ref = np.where(np.isinf(ref), -1, ref).astype(np.int64)
        assert np.array_equal(oracle.wmssp(g, w, s, threads=4), ref)


@pytest.mark.parametrize("name", ["rmat12", "grid128", "uniform4096"])
def test_unit_weights_are_hop_counts(name):
    g, src = gg.load_config(name)
    w = np.ones(g.m, np.int32)
    assert np.array_equal(oracle.wmssp(g, w, src[:8], threads=4),
                          oracle.mssp(g, src[:8]).astype(np.int64))


def test_closed_forms():
    # directed path 0 -> 1 -> ... -> 9 with weights 1..9: prefix sums
    n = 10
    g = gg.gen_edges(n, [(i, i + 1) for i in range(n - 1)])
    w = np.arange(1, n, dtype=np.int32)
    assert oracle.wsssp(g, w, 0).tolist() == np.concatenate([[0], np.cumsum(w)]).tolist()
    assert oracle.wsssp(g, w, 5).tolist() == [-1] * 5 + [0, 6, 13, 21, 30]
    # a heavy direct edge loses to a light detour: 0 -> 2 (10) vs 0 -> 1 -> 2 (3 + 4)
    g = gg.gen_edges(3, [(0, 1), (0, 2), (1, 2)])
    order = {(0, 1): 3, (0, 2): 10, (1, 2): 4}
    src = np.repeat(np.arange(3), np.diff(g.row_ptr))
    w = np.array([order[(int(a), int(b))] for a, b in zip(src, g.col)], np.int32)
    assert oracle.wsssp(g, w, 0).tolist() == [0, 3, 7]
    # zero weights: everything reachable is at distance 0
    g, _ = gg.load_config("grid128")
    z = np.zeros(g.m, np.int32)
    d = oracle.wsssp(g, z, 0)
    assert set(np.unique(d).tolist()) <= {-1, 0}
    assert np.array_equal(d >= 0, oracle.forward_reachable(g, 0))


def test_negative_weights_refused():
    g = gg.gen_edges(3, [(0, 1), (1, 2)])
    with pytest.raises(ValueError):
        oracle.wsssp(g, np.array([1, -1], np.int32), 0)


@pytest.mark.parametrize("name", ["rmat12", "grid128", "grid128ns"])
def test_weighted_invariants_on_workloads(name):
    g, src = gg.load_config(name)
    w = gg.gen_weights(g, 1, 100, seed=3, symmetric=True)
    for s in src[:4]:
        oracle.check_weighted_invariants(g, w, int(s), oracle.wsssp(g, w, int(s)))


def _dijkstra_variant(g, w, s, mistake):
    """Python Dijkstra with one deliberate slip; used only to show the pins bite."""
    import heapq
    dist = np.full(g.n, -1, np.int64)
    dist[s] = 0
    h = [(0, s)]
    done = np.zeros(g.n, bool)
    while h:
        d, u = heapq.heappop(h)
        if done[u]:
            continue
        done[u] = True
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[e])
            if mistake == "hops":
                nd = d + 1
            elif mistake == "max_weight":
                nd = max(d, int(w[e]))
            else:
                nd = d + int(w[e])
            if mistake == "first_found":
                if dist[v] == -1:
                    dist[v] = nd
                    heapq.heappush(h, (nd, v))
            elif dist[v] == -1 or nd < dist[v]:
                dist[v] = nd
                heapq.heappush(h, (nd, v))
    return dist


@pytest.mark.parametrize("mistake", ["hops", "max_weight", "first_found"])
def test_pins_detect_planted_mistakes(mistake):
    caught = False
    for i, g, w in _tiny_weighted(count=80, seed=11):
        if g.n < 4:
            continue
        fw = oracle.floyd_warshall_weighted(g, w)
        bad = np.stack([_dijkstra_variant(g, w, s, mistake) for s in range(g.n)])
        if not np.array_equal(bad, fw):
            caught = True
            break
    assert caught, f"planted mistake {mistake!r} was not caught"
    for i, g, w in _tiny_weighted(count=20, seed=11):
        fw = oracle.floyd_warshall_weighted(g, w)
        good = np.stack([_dijkstra_variant(g, w, s, "none") for s in range(g.n)])
        assert np.array_equal(good, fw)


def test_weighted_invariant_checker_detects_corruption():
    g, src = gg.load_config("rmat12")
    w = gg.gen_weights(g, 1, 50, seed=4, symmetric=True)
    s = int(src[0])
    d = oracle.wsssp(g, w, s)
    oracle.check_weighted_invariants(g, w, s, d)
    far = np.nonzero(d > 10)[0]
    for mutate in (lambda x: x.__setitem__(far[0], x[far[0]] + 1),
                   lambda x: x.__setitem__(far[1], x[far[1]] - 1),
                   lambda x: x.__setitem__(far[2], -1)):
        bad = d.copy()
        mutate(bad)
        with pytest.raises(AssertionError):
            oracle.check_weighted_invariants(g, w, s, bad)
