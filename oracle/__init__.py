"""CPU oracle for DAWN's results — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.

Contents
--------
``sssp``, ``mssp``, ``largest_wcc``
    ctypes wrappers over ``bfs_oracle.c``: a FIFO-queue BFS per source (the
    general BFS of the paper's Section 3.5, Algorithm 3, with -1 for "not
    reached") and an undirected-sweep WCC.
``floyd_warshall``
    All-pairs hop distances by the Floyd–Warshall recurrence, O(n^3): an
    independent algorithm used to pin the BFS on tiny graphs.
``bool_power_distances``
    Theorem 1 of the paper (Section 3.1) written out: dist(i, j) is the
    smallest k >= 1 with (A^k)_ij != 0 for i != j; Lemma 1 says (A^k)_ij
    counts length-k paths, so the boolean power suffices.
``wsssp``, ``wmssp``
    Weighted graphs (the (min, +) extension the paper leaves to future work):
    Dijkstra's algorithm with a binary heap over non-negative integer weights
    (``dijkstra_oracle.c``), int64 distances, -1 where unreachable.
``floyd_warshall_weighted``, ``check_weighted_invariants``
    Their pins: the weighted Floyd–Warshall recurrence on tiny graphs, and the
    properties of exact weighted distances at any size.
``check_invariants``
    Properties that hold at any size: dist[s] = 0; on every edge (u, v) with
    u reached, 0 <= dist[v] <= dist[u] + 1 (Fact 1, Section 3.1); every
    reached v != s has an in-neighbour at dist[v] - 1; the reached set equals
    forward reachability found by an independent depth-first search.

Every function here is "parity pinned" by ``tests/test_oracle.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_I32P)


def lib():
    """Load ``liboracle.so``, compiling it first only when it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oracle_sssp.argtypes = [ctypes.c_int32, _I32P, _I32P, ctypes.c_int32, _I32P]
        L.oracle_mssp.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P, ctypes.c_int32,
                                  _I32P, ctypes.c_int32]
        L.oracle_largest_wcc.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P, _I32P]
        L.oracle_wsssp.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P, ctypes.c_int32, _I64P]
        L.oracle_wmssp.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P, _I32P, ctypes.c_int32,
                                   _I64P, ctypes.c_int32]
        for f in (L.oracle_sssp, L.oracle_mssp, L.oracle_largest_wcc, L.oracle_wsssp,
                  L.oracle_wmssp):
            f.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return rp, col


def sssp(g, s: int) -> np.ndarray:
    """Shortest-path lengths from ``s`` (int32, -1 where unreachable)."""
    rp, col = _csr(g)
    dist = np.empty(g.n, dtype=np.int32)
    if lib().oracle_sssp(g.n, _ptr(rp), _ptr(col), int(s), _ptr(dist)) != 0:
        raise ValueError("oracle_sssp: bad argument")
    return dist


def mssp(g, sources, threads: int = 1) -> np.ndarray:
    """Row r = ``sssp(g, sources[r])``; computed with ``threads`` POSIX threads."""
    rp, col = _csr(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = src.size
    dist = np.empty((k, g.n), dtype=np.int32)
    if k == 0:
        return dist
    if lib().oracle_mssp(g.n, _ptr(rp), _ptr(col), _ptr(src), k, _ptr(dist),
                         int(threads)) != 0:
        raise ValueError("oracle_mssp: bad argument")
    return dist


def _weights(g, weight):
    w = np.ascontiguousarray(weight, dtype=np.int32)
    if w.shape != (g.m,):
        raise ValueError("one weight per CSR entry")
    if w.size == 0:
        w = np.zeros(1, dtype=np.int32)
    return w


def wsssp(g, weight, s: int) -> np.ndarray:
    """Weighted shortest-path lengths from ``s`` (int64, -1 where unreachable).

    ``weight[e]`` belongs to CSR entry e; weights must be >= 0."""
    rp, col = _csr(g)
    w = _weights(g, weight)
    dist = np.empty(g.n, dtype=np.int64)
    if lib().oracle_wsssp(g.n, _ptr(rp), _ptr(col), _ptr(w), int(s),
                          dist.ctypes.data_as(_I64P)) != 0:
        raise ValueError("oracle_wsssp: bad argument (negative weight?)")
    return dist


def wmssp(g, weight, sources, threads: int = 1) -> np.ndarray:
    """Row r = ``wsssp(g, weight, sources[r])``, on ``threads`` POSIX threads."""
    rp, col = _csr(g)
    w = _weights(g, weight)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    dist = np.empty((src.size, g.n), dtype=np.int64)
    if src.size == 0:
        return dist
    if lib().oracle_wmssp(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(src), src.size,
                          dist.ctypes.data_as(_I64P), int(threads)) != 0:
        raise ValueError("oracle_wmssp: bad argument")
    return dist


def floyd_warshall_weighted(g, weight) -> np.ndarray:
    """All-pairs weighted distances by d[i,j] = min(d[i,j], d[i,k] + d[k,j]).

    Tiny graphs only; a repeated edge keeps its lightest weight.  int64 with
    -1 for unreachable pairs and 0 on the diagonal."""
    n = g.n
    inf = np.int64(1) << 60
    d = np.full((n, n), inf, dtype=np.int64)
    for u in range(n):
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[e])
            d[u, v] = min(d[u, v], int(weight[e]))
    np.fill_diagonal(d, 0)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return np.where(d >= inf, -1, d)


def check_weighted_invariants(g, weight, s: int, dist: np.ndarray,
                              reach: np.ndarray | None = None) -> None:
    """Raise AssertionError unless ``dist`` holds exact weighted distances from s:
    dist[s] = 0; every edge (u, v, w) with u reached has v reached and
    dist[v] <= dist[u] + w; every reached v != s has an in-edge with
    dist[u] + w = dist[v] (a tight predecessor); the reached set equals
    forward reachability.  With positive weights these fix the distances
    (following tight in-edges from any reached node strictly lowers the value
    and so ends at s); a cycle of zero-weight edges could hold too small a
    value, so zero weights are pinned by Dijkstra against Floyd–Warshall."""
    dist = np.asarray(dist, dtype=np.int64)
    w = np.asarray(weight, dtype=np.int64)
    n = g.n
    assert dist.shape == (n,) and dist[s] == 0
    assert (dist >= -1).all()
    deg = np.diff(g.row_ptr.astype(np.int64))
    src = np.repeat(np.arange(n), deg)
    dst = g.col.astype(np.int64)
    du, dv = dist[src], dist[dst]
    r = du >= 0
    assert (dv[r] >= 0).all(), "target of a reached node must be reached"
    assert (dv[r] <= du[r] + w[r]).all(), "dist[v] <= dist[u] + w(u, v)"
    tight = np.zeros(n, dtype=bool)
    ok = r & (dv == du + w)
    tight[dst[ok]] = True
    need = dist >= 0
    need[s] = False
    assert tight[need].all(), "reached node without a tight in-edge"
    if reach is None:
        reach = forward_reachable(g, s)
    assert np.array_equal(dist >= 0, reach), "reached set != forward reachability"


def largest_wcc(g) -> np.ndarray:
    """Ascending node ids of the largest WCC (ties: the one holding the smallest id)."""
    rp, col = _csr(g)
    out = np.empty(g.n, dtype=np.int32)
    cnt = np.zeros(1, dtype=np.int32)
    if lib().oracle_largest_wcc(g.n, _ptr(rp), _ptr(col), _ptr(out), _ptr(cnt)) != 0:
        raise ValueError("oracle_largest_wcc: bad argument")
    return out[: int(cnt[0])].copy()


def adjacency(g) -> np.ndarray:
    """Dense 0/1 adjacency matrix ``A[u, v] = 1`` iff edge u -> v (tiny graphs only)."""
    a = np.zeros((g.n, g.n), dtype=np.int64)
    for u in range(g.n):
        a[u, g.col[g.row_ptr[u]:g.row_ptr[u + 1]]] = 1
    return a


def floyd_warshall(a: np.ndarray) -> np.ndarray:
    """Hop distances by the Floyd–Warshall recurrence d[i,j] = min(d[i,j], d[i,k] + d[k,j]).

    ``a`` is a dense 0/1 adjacency matrix.  Returns int32 with -1 for
    unreachable pairs and 0 on the diagonal.
    """
    n = a.shape[0]
    inf = np.int64(n + 1)
    d = np.where(a != 0, 1, inf).astype(np.int64)
    np.fill_diagonal(d, 0)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    out = np.where(d >= inf, -1, d)
    return out.astype(np.int32)


def bool_power_distances(a: np.ndarray) -> np.ndarray:
    """Theorem 1: dist(i, j) = min{k >= 1 : (A^k)_ij != 0} for i != j; 0 on the diagonal.

    Boolean powers are formed by repeated products with A (a library matmul),
    clipped to 0/1 after each step; k runs to n - 1, the longest possible
    shortest path.  -1 where no power is non-zero.
    """
    n = a.shape[0]
    a = (a != 0).astype(np.int64)
    dist = np.full((n, n), -1, dtype=np.int32)
    np.fill_diagonal(dist, 0)
    p = a.copy()
    for k in range(1, n):
        hit = (p != 0) & (dist == -1)
        dist[hit] = k
        p = ((p @ a) != 0).astype(np.int64)
    return dist


def forward_reachable(g, s: int) -> np.ndarray:
    """Boolean mask of nodes reachable from ``s`` by an iterative depth-first search."""
    seen = np.zeros(g.n, dtype=bool)
    stack = [int(s)]
    seen[s] = True
    rp, col = g.row_ptr, g.col
    while stack:
        u = stack.pop()
        for v in col[rp[u]:rp[u + 1]]:
            if not seen[v]:
                seen[v] = True
                stack.append(int(v))
    return seen


def check_invariants(g, s: int, dist: np.ndarray, reach: np.ndarray | None = None) -> None:
    """Raise AssertionError unless ``dist`` satisfies the shortest-path invariants."""
    dist = np.asarray(dist, dtype=np.int64)
    n = g.n
    assert dist.shape == (n,)
    assert dist[s] == 0, "dist[s] must be 0"
    assert (dist >= -1).all()
    others = np.arange(n) != s
    assert (dist[others] != 0).all(), "only the source has distance 0"
    deg = np.diff(g.row_ptr.astype(np.int64))
    src = np.repeat(np.arange(n), deg)
    dst = g.col.astype(np.int64)
    du, dv = dist[src], dist[dst]
    reached_edge = du >= 0
    # Fact 1 / edge relaxation: a reached u makes its target reached within one step
    assert (dv[reached_edge] >= 0).all(), "target of a reached node must be reached"
    assert (dv[reached_edge] <= du[reached_edge] + 1).all(), "dist[v] <= dist[u] + 1"
    # every reached v != s has a predecessor one level closer
    has_parent = np.zeros(n, dtype=bool)
    ok = reached_edge & (dv == du + 1)
    has_parent[dst[ok]] = True
    need = (dist > 0)
    assert has_parent[need].all(), "reached node without an in-neighbour at dist-1"
    if reach is None:
        reach = forward_reachable(g, s)
    assert np.array_equal(dist >= 0, reach), "reached set != forward reachability"
