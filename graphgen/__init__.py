"""Seeded synthetic graphs and source sets (inputs only).

This module is shared by the CPU oracle side (tests) and by the GPU path
(tests, bench).  It builds edge lists and packs them into int32 CSR; it holds
no shortest-path arithmetic.  The paper's 66 SuiteSparse/Gunrock graphs are not
available, so seeded stand-ins take their place (Section 4.1 of the paper
describes the originals):

* directed uniform-random graphs (small, CPU-checkable);
* R-MAT graphs (scale-free, like the paper's social and web graphs);
* damaged 2-D grids with a few random shortcuts (high-diameter, like the
  paper's road networks).

Every generator draws from numpy's PCG64 (``numpy.random.default_rng``) with
an explicit seed, so the same call always yields the same CSR.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph", "to_csr", "gen_uniform", "gen_rmat", "gen_grid", "gen_edges",
    "gen_islands", "largest_wcc_nodes", "sample_sources", "CONFIGS", "load_config",
    "reach_edges_from_dist", "gen_weights",
]


@dataclass
class Graph:
    """An int32 CSR graph: row ``u`` of ``col`` holds the out-neighbours of ``u``."""

    n: int
    row_ptr: np.ndarray          # int32[n+1]
    col: np.ndarray              # int32[m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


# ---------------------------------------------------------------------------
# CSR packing
# ---------------------------------------------------------------------------

def to_csr(n: int, src, dst, *, symmetrize: bool = False, drop_self: bool = True,
           dedupe: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """Pack an edge list into int32 CSR with rows sorted by target id.

    ``symmetrize`` adds the reverse of every edge; ``drop_self`` removes
    ``u -> u``; ``dedupe`` keeps one copy of each ``(u, v)``.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if symmetrize:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    if drop_self:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    key = src * np.int64(n) + dst
    key = np.unique(key) if dedupe else np.sort(key, kind="stable")
    s = (key // n).astype(np.int64)
    d = (key % n).astype(np.int32)
    counts = np.bincount(s, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("edge count exceeds int32")
    return row_ptr.astype(np.int32), np.ascontiguousarray(d)


def gen_edges(n: int, pairs, *, symmetrize=False, drop_self=True, dedupe=True,
              name="custom") -> Graph:
    """Build a Graph from an explicit list of ``(u, v)`` pairs (tests)."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    rp, col = to_csr(n, pairs[:, 0], pairs[:, 1], symmetrize=symmetrize,
                     drop_self=drop_self, dedupe=dedupe)
    return Graph(n, rp, col, name)


# ---------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------

def gen_uniform(n: int, m: int, seed: int) -> Graph:
    """Directed graph with exactly ``m`` distinct non-loop edges.

    Endpoints are drawn uniformly; self-loops and repeats are dropped and more
    pairs are drawn until ``m`` distinct edges remain (first occurrences in
    draw order are kept, the first ``m`` of them form the graph).
    """
    if m > n * (n - 1):
        raise ValueError("m too large for a simple directed graph")
    rng = np.random.default_rng(seed)
    keys = np.empty(0, dtype=np.int64)
    while True:
        need = m - keys.size
        batch = max(1024, int(need * 1.2) + 64)
        u = rng.integers(0, n, size=batch, dtype=np.int64)
        v = rng.integers(0, n, size=batch, dtype=np.int64)
        k = u * n + v
        k = k[u != v]
        allk = np.concatenate([keys, k])
        _, first = np.unique(allk, return_index=True)
        keys = allk[np.sort(first)]
        if keys.size >= m:
            keys = keys[:m]
            break
    rp, col = to_csr(n, keys // n, keys % n)
    return Graph(n, rp, col, f"uniform-n{n}-m{m}", {"seed": seed, "kind": "uniform"})


def gen_rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
             symmetrize=True, permute=True) -> Graph:
    """R-MAT graph on ``2**scale`` nodes from ``edge_factor * 2**scale`` draws.

    Each draw picks one of the four quadrants with probabilities a, b, c, d at
    every one of the ``scale`` bit levels (no per-level noise).  Node ids are
    then relabelled by one seeded random permutation, the edge set is
    symmetrised, self-loops are dropped and repeats removed.
    """
    n = 1 << scale
    draws = edge_factor * n
    rng = np.random.default_rng(seed)
    src = np.zeros(draws, dtype=np.int64)
    dst = np.zeros(draws, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for _ in range(scale):
        r = rng.random(draws)
        sbit = r >= ab                           # quadrants c or d: lower half
        dbit = ((r >= a) & (r < ab)) | (r >= abc)  # quadrants b or d: right half
        src = (src << 1) | sbit
        dst = (dst << 1) | dbit
        del r, sbit, dbit
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src, dst = perm[src], perm[dst]
    rp, col = to_csr(n, src, dst, symmetrize=symmetrize)
    return Graph(n, rp, col, f"rmat-s{scale}-ef{edge_factor}",
                 {"seed": seed, "kind": "rmat", "a": a, "b": b, "c": c,
                  "symmetric": symmetrize})


def gen_grid(k: int, seed: int, delete_frac=0.05, shortcut_frac=0.001) -> Graph:
    """Undirected ``k x k`` 4-neighbour grid, damaged, with random shortcuts.

    Node id is ``row * k + col``.  Of the ``E = 2k(k-1)`` grid edges exactly
    ``floor(delete_frac * E)`` are removed (uniform, without replacement) and
    ``floor(shortcut_frac * E)`` undirected shortcuts with uniform endpoints
    are added; the result is symmetrised, de-duplicated and loop-free.
    """
    n = k * k
    rng = np.random.default_rng(seed)
    r, c = np.meshgrid(np.arange(k, dtype=np.int64), np.arange(k, dtype=np.int64),
                       indexing="ij")
    hs = (r[:, :-1] * k + c[:, :-1]).ravel()
    hd = hs + 1
    vs = (r[:-1, :] * k + c[:-1, :]).ravel()
    vd = vs + k
    es = np.concatenate([hs, vs])
    ed = np.concatenate([hd, vd])
    E = es.size
    assert E == 2 * k * (k - 1)
    ndel = int(np.floor(delete_frac * E))
    if ndel:
        drop = rng.choice(E, size=ndel, replace=False)
        keep = np.ones(E, dtype=bool)
        keep[drop] = False
        es, ed = es[keep], ed[keep]
    nsc = int(np.floor(shortcut_frac * E))
    if nsc:
        su = rng.integers(0, n, size=nsc, dtype=np.int64)
        sv = rng.integers(0, n, size=nsc, dtype=np.int64)
        es, ed = np.concatenate([es, su]), np.concatenate([ed, sv])
    rp, col = to_csr(n, es, ed, symmetrize=True)
    return Graph(n, rp, col, f"grid-{k}-del{delete_frac}-sc{shortcut_frac}",
                 {"seed": seed, "kind": "grid", "k": k, "deleted": ndel,
                  "shortcuts": nsc, "symmetric": True})


# ---------------------------------------------------------------------------
# Source selection
# ---------------------------------------------------------------------------

def gen_islands(count: int, min_size: int, max_size: int, degree: int, seed: int) -> Graph:
    """Disjoint union of ``count`` small symmetric random graphs.

    Component sizes are log-uniform in [min_size, max_size]; each component
    has a path through its nodes (so it is connected) plus ``degree / 2 *
    size`` uniform pairs, symmetrised, without self-loops or repeats; node
    ids are then relabelled by one seeded permutation.
    """
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(min_size), np.log(max_size + 1), size=count)))
    sizes = sizes.astype(np.int64)
    src, dst, base = [], [], 0
    for sz in sizes:
        chain = np.arange(sz - 1, dtype=np.int64)
        extra = rng.integers(0, sz, size=(int(degree // 2 * sz), 2), dtype=np.int64)
        src += [chain + base, extra[:, 0] + base]
        dst += [chain + 1 + base, extra[:, 1] + base]
        base += int(sz)
    n = base
    perm = rng.permutation(n).astype(np.int64)
    u = perm[np.concatenate(src)]
    v = perm[np.concatenate(dst)]
    rp, col = to_csr(n, u, v, symmetrize=True)
    return Graph(n, rp, col, f"islands-{count}", {"seed": seed, "kind": "islands"})


def largest_wcc_nodes(g: Graph) -> np.ndarray:
    """Ascending node ids of the largest weakly connected component.

    Used only to choose sources.  Ties between equally large components go to
    the one that holds the smallest node id.
    """
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    a = csr_matrix((np.ones(g.m, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    ncomp, labels = connected_components(a, directed=True, connection="weak")
    sizes = np.bincount(labels, minlength=ncomp)
    minid = np.full(ncomp, g.n, dtype=np.int64)
    np.minimum.at(minid, labels, np.arange(g.n))
    best = max(range(ncomp), key=lambda c: (sizes[c], -minid[c]))
    return np.nonzero(labels == best)[0].astype(np.int32)


def gen_weights(g: Graph, lo: int, hi: int, seed: int, symmetric: bool = False) -> np.ndarray:
    """Seeded integer edge weights, uniform in [lo, hi], one per CSR entry.

    With ``symmetric`` the two directions of an edge get the same weight (a
    hash of the unordered pair and the seed picks it), as on a road network.
    The paper's weighted experiments are future work, so this is a plain
    stand-in: uniform weights on the same synthetic graphs."""
    if hi < lo or lo < 0:
        raise ValueError("need 0 <= lo <= hi")
    span = np.uint64(hi - lo + 1)
    if not symmetric:
        rng = np.random.default_rng(seed)
        return rng.integers(lo, hi + 1, size=g.m).astype(np.int32)
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr.astype(np.int64)))
    dst = g.col.astype(np.uint64)
    a, b = np.minimum(src, dst), np.maximum(src, dst)
    with np.errstate(over="ignore"):
        x = (a * np.uint64(0x9E3779B97F4A7C15)) ^ (b + np.uint64(seed) * np.uint64(0xBF58476D1CE4E5B9))
        x ^= x >> np.uint64(31)
        x *= np.uint64(0x94D049BB133111EB)
        x ^= x >> np.uint64(29)
    return (np.uint64(lo) + x % span).astype(np.int32)


def sample_sources(pool, k: int, seed: int) -> np.ndarray:
    """``k`` distinct sources drawn uniformly from ``pool`` (ints or an array)."""
    rng = np.random.default_rng(seed)
    pool = np.arange(pool, dtype=np.int32) if np.isscalar(pool) else np.asarray(pool, np.int32)
    if k > pool.size:
        raise ValueError("not enough nodes to sample from")
    return np.ascontiguousarray(rng.choice(pool, size=k, replace=False).astype(np.int32))


def reach_edges_from_dist(g: Graph, dist: np.ndarray) -> int:
    """Sum of out-degrees over the nodes a distance row reaches (dist >= 0).

    This is the traversal-count numerator used for GTEPS (edges out of every
    reached node, counted as directed CSR edges).
    """
    deg = g.out_degree()
    d = np.asarray(dist)
    if d.ndim == 1:
        return int(deg[d >= 0].sum())
    return int(((d >= 0).astype(np.int64) @ deg).sum())


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    # small, CPU-checkable: directed uniform random, 8 sources over [0, n)
    "uniform4096": dict(kind="uniform", n=4096, m=32768, seed=1, src_seed=101,
                        k=8, from_wcc=False),
    # R-MAT scale 20, edge factor 16, 64 sources from the largest WCC
    "rmat20": dict(kind="rmat", scale=20, ef=16, seed=2, src_seed=102, k=64,
                   from_wcc=True),
    # 2048^2 damaged grid with shortcuts, 16 sources from the largest WCC
    "grid2048": dict(kind="grid", k=2048, seed=3, src_seed=103, k_src=16,
                     from_wcc=True, delete=0.05, shortcut=0.001),
    # same grid without shortcuts (thousands of levels)
    "grid2048ns": dict(kind="grid", k=2048, seed=3, src_seed=103, k_src=16,
                       from_wcc=True, delete=0.05, shortcut=0.0),
    # batched: R-MAT scale 18, 4096 sources in one launch
    "rmat18": dict(kind="rmat", scale=18, ef=16, seed=4, src_seed=104, k=4096,
                   from_wcc=True),
    # APSP over the largest WCC of R-MAT scale 14
    "rmat14": dict(kind="rmat", scale=14, ef=16, seed=5, src_seed=105, k=0,
                   from_wcc=True),
    # serving graphs
    "rmat16": dict(kind="rmat", scale=16, ef=16, seed=6, src_seed=106, k=0,
                   from_wcc=True),
    "grid1024": dict(kind="grid", k=1024, seed=7, src_seed=107, k_src=0,
                     from_wcc=True, delete=0.05, shortcut=0.001),
    # many small components (log-uniform 16 .. 2048 nodes), 64 sources over all nodes
    "islands": dict(kind="islands", count=512, min_size=16, max_size=2048, degree=8, seed=10,
                    src_seed=110, k=64, from_wcc=False),
    # reduced-size variants for quick tests
    "rmat12": dict(kind="rmat", scale=12, ef=16, seed=8, src_seed=108, k=64,
                   from_wcc=True),
    "grid128": dict(kind="grid", k=128, seed=9, src_seed=109, k_src=16,
                    from_wcc=True, delete=0.05, shortcut=0.001),
    "grid128ns": dict(kind="grid", k=128, seed=9, src_seed=109, k_src=16,
                      from_wcc=True, delete=0.05, shortcut=0.0),
}


def _cache_dir() -> str | None:
    d = os.environ.get("DAWN_GRAPH_CACHE")
    if d == "":
        return None
    if d is None:
        d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         ".graph_cache")
    return d


def _build(cfg: dict) -> Graph:
    kind = cfg["kind"]
    if kind == "uniform":
        return gen_uniform(cfg["n"], cfg["m"], cfg["seed"])
    if kind == "rmat":
        return gen_rmat(cfg["scale"], cfg["ef"], cfg["seed"])
    if kind == "grid":
        return gen_grid(cfg["k"], cfg["seed"], cfg["delete"], cfg["shortcut"])
    if kind == "islands":
        return gen_islands(cfg["count"], cfg["min_size"], cfg["max_size"], cfg["degree"],
                           cfg["seed"])
    raise ValueError(kind)


def load_config(name: str, use_cache: bool = True) -> tuple[Graph, np.ndarray]:
    """Return ``(graph, sources)`` for a named workload.

    Graphs are cached as ``.npz`` keyed by a hash of the config, so the same
    config always maps to the same file; a missing cache is rebuilt.
    """
    cfg = CONFIGS[name]
    key = hashlib.sha1(json.dumps(cfg, sort_keys=True).encode()).hexdigest()[:12]
    cdir = _cache_dir() if use_cache else None
    path = os.path.join(cdir, f"{name}-{key}.npz") if cdir else None
    g = None
    if path and os.path.exists(path):
        z = np.load(path)
        g = Graph(int(z["n"]), z["row_ptr"], z["col"], name,
                  json.loads(str(z["meta"])))
        wcc = z["wcc"]
    if g is None:
        g = _build(cfg)
        g.name = name
        wcc = largest_wcc_nodes(g) if cfg.get("from_wcc") else np.arange(g.n, dtype=np.int32)
        if path:
            os.makedirs(cdir, exist_ok=True)
            tmp = path + ".tmp.npz"
            np.savez(tmp, n=g.n, row_ptr=g.row_ptr, col=g.col, wcc=wcc,
                     meta=json.dumps(g.meta))
            os.replace(tmp, path)
    g.meta["wcc_size"] = int(wcc.size)
    k = cfg.get("k", cfg.get("k_src", 0))
    if k:
        pool = wcc if cfg.get("from_wcc") else g.n
        src = sample_sources(pool, k, cfg["src_seed"])
    else:
        src = np.empty(0, dtype=np.int32)
    g.meta["wcc_nodes"] = wcc
    return g, src
