"""Single-source parity: the HIP path through the C ABI vs the CPU oracle, bit for bit.

Distances are integers, so the bar is exact equality (tolerance 0).  Every
forced variant (driver, direction, workgroup size, big-degree threshold,
pull lane budget) must give the oracle's row; the per-level counters must
match the oracle's distance histogram.
"""
import itertools
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from conftest import load_golden
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _check_row(g, s, got, stats=None, all_push=False):
    want = oracle.sssp(g, int(s))
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"source {s}: {bad.size} mismatches, first at {bad[:5]}: "
                             f"got {got[bad[:5]]} want {want[bad[:5]]}")
    if stats is not None:
        lv = int(want.max()) + 1
        assert stats["levels"] == lv
        deg = g.out_degree()
        assert stats["reached"] == int((want >= 0).sum())
        assert stats["source_edges"] == int(deg[want >= 0].sum())
        if "frontier_sizes" in stats:
            hist = np.bincount(want[want >= 0], minlength=lv)
            assert stats["frontier_sizes"] == hist[: len(stats["frontier_sizes"])].tolist()
        if all_push:
            # every out-edge of every reached node is examined exactly once
            assert stats["edges_examined"] == int(deg[want >= 0].sum())
    return want


VARIANTS = [
    dict(driver=1, direction=3), dict(driver=1, direction=1), dict(driver=1, direction=2),
    dict(driver=2, direction=3), dict(driver=2, direction=1), dict(driver=2, direction=2),
    dict(driver=3, direction=3, graph_levels=4), dict(driver=3, direction=1, graph_levels=16),
    dict(driver=4, direction=3, graph_levels=6), dict(driver=4, direction=2, graph_levels=2),
    dict(driver=1, direction=3, block=512), dict(driver=1, direction=3, block=1024),
    dict(driver=1, direction=1, big_degree=64), dict(driver=2, direction=1, big_degree=64, block=1024),
    dict(driver=1, direction=2, pull_lane_edges=1), dict(driver=1, direction=3, alpha=1e6, beta=1e-3),
    dict(driver=1, direction=3, blocks_per_cu=1), dict(driver=1, direction=3, small_n=1 << 30),
    # one workgroup runs the small push levels: never, always, and always with
    # the graph driver and the smallest workgroup
    dict(driver=3, direction=3, small_frontier_edges=-1),
    dict(driver=2, direction=1, small_frontier_edges=1 << 30),
    dict(driver=4, direction=3, graph_levels=6, small_frontier_edges=1 << 30, block=256),
    dict(driver=3, direction=3, graph_levels=4, small_frontier_edges=64),
    # medium push levels on a few workgroups of a launch: the default bound,
    # every push level past the one-workgroup ones (two workgroups), with the
    # one-workgroup levels off, and under the per-level and graph drivers
    dict(driver=3, direction=3, medium_edges=65536),
    dict(driver=3, direction=1, graph_levels=4, medium_edges=1 << 30, medium_groups=2),
    dict(driver=3, direction=3, medium_edges=1 << 30, small_frontier_edges=-1, medium_groups=64),
    dict(driver=2, direction=1, medium_edges=4096, medium_groups=8, block=1024),
    dict(driver=4, direction=3, graph_levels=6, medium_edges=65536, block=256),
]


@pytest.fixture
def restore(ctx):
    touched = []

    def _set(graph, **kw):
        if graph not in [t[0] for t in touched]:
            touched.append((graph, D.dawn_get_params(ctx, graph)))
        return D.dawn_set_params(ctx, graph, **kw)
    yield _set
    for graph, p in touched:
        D.dawn_set_params(ctx, graph, **p)


@pytest.mark.parametrize("name", ["uniform4096", "rmat12", "grid128", "grid128ns"])
@pytest.mark.parametrize("vi", range(len(VARIANTS)))
def test_variants_bit_exact(ctx, upload, restore, name, vi):
    h, g, src = upload(name)
    v = VARIANTS[vi]
    _say(f"[sssp] {name} variant {v}")
    restore(h, **v)
    for s in src[:4]:
        got, st = D.dawn_sssp(ctx, h, int(s), frontier_cap=4096)
        _check_row(g, s, got, st, all_push=(v.get("direction") == 1))
        dirs = st["directions"]
        if v.get("direction") == 1:
            assert set(dirs[1:]) <= {1}
        if v.get("direction") == 2:
            assert set(dirs[1:]) <= {2}


def test_all_sources_default(ctx, upload):
    h, g, src = upload("uniform4096")
    for s in src:
        got, st = D.dawn_sssp(ctx, h, int(s), frontier_cap=64)
        _check_row(g, s, got, st)


@pytest.mark.parametrize("name", ["hand_directed10.txt", "petersen.txt"])
def test_golden_graphs(ctx, name):
    n, edges, rows = load_golden(name)
    g = gg.gen_edges(n, edges, drop_self=False, dedupe=False)
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        for s, want in rows.items():
            for direction in (1, 2, 3):
                D.dawn_set_params(ctx, h, direction=direction)
                got, _ = D.dawn_sssp(ctx, h, s)
                assert np.array_equal(got, want), (name, s, direction)
    finally:
        D.dawn_graph_release(ctx, h)


def test_tiny_random_graphs(ctx):
    rng = np.random.default_rng(7)
    for i in range(40):
        n = int(rng.integers(1, 200))
        m = int(rng.integers(0, 4 * n))
        e = rng.integers(0, n, size=(m, 2))
        g = gg.gen_edges(n, e, symmetrize=bool(i % 2), drop_self=False, dedupe=bool(i % 3))
        h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        try:
            for direction, driver in itertools.product((1, 2, 3), (1, 2)):
                D.dawn_set_params(ctx, h, direction=direction, driver=driver)
                for s in sorted(set(rng.integers(0, n, size=3).tolist())):
                    got, st = D.dawn_sssp(ctx, h, s, frontier_cap=256)
                    _check_row(g, s, got, st, all_push=(direction == 1))
        finally:
            D.dawn_graph_release(ctx, h)


def test_edge_cases(ctx):
    # single node, no edges
    g = gg.gen_edges(1, np.zeros((0, 2), np.int64))
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    got, st = D.dawn_sssp(ctx, h, 0)
    assert got.tolist() == [0] and st["levels"] == 1
    D.dawn_graph_release(ctx, h)
    # out-degree-0 source in a star; a hub whose out-degree exceeds every chunk size
    n = 5000
    g = gg.gen_edges(n, [(0, i) for i in range(1, n)] + [(i, 0) for i in range(1, 50)])
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        for s in (0, 7, 60):
            for direction in (1, 2, 3):
                D.dawn_set_params(ctx, h, direction=direction, big_degree=64)
                got, st = D.dawn_sssp(ctx, h, s, frontier_cap=16)
                _check_row(g, s, got, st, all_push=(direction == 1))
    finally:
        D.dawn_graph_release(ctx, h)
    # n not a multiple of 64, a long directed path (many levels)
    n = 3001
    g = gg.gen_edges(n, [(i, i + 1) for i in range(n - 1)])
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        for driver in (1, 2, 3, 4):
            D.dawn_set_params(ctx, h, driver=driver, graph_levels=64)
            got, st = D.dawn_sssp(ctx, h, 5, frontier_cap=8)
            _check_row(g, 5, got, st)
            assert st["levels"] == n - 5
    finally:
        D.dawn_graph_release(ctx, h)


def test_device_output_torch(ctx, upload):
    import torch
    h, g, src = upload("rmat12")
    out = torch.full((3, g.n), 7, dtype=torch.int32, device="cuda")
    for r, s in enumerate(src[:3]):
        D.dawn_sssp(ctx, h, int(s), out=out[r])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for r, s in enumerate(src[:3]):
        _check_row(g, s, got[r])


def test_device_output_any_alignment(ctx):
    """Device rows that start at every 4-byte offset within 16 bytes, on a
    graph whose node count is not a multiple of 4: each row is exact and
    nothing around it is written."""
    import torch
    g = gg.gen_uniform(1003, 8000, seed=17)
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        flat = torch.empty((g.n + 8,), dtype=torch.int32, device="cuda")
        for off in range(4):
            for s in (0, 1, 2, 3, 500, g.n - 1):
                flat.fill_(7)
                row = flat[off: off + g.n]
                D.dawn_sssp(ctx, h, s, out=row)
                torch.cuda.synchronize()
                _check_row(g, s, row.cpu().numpy())
                # nothing outside the row is written
                rest = torch.cat([flat[:off], flat[off + g.n:]])
                assert int(rest.ne(7).sum()) == 0
    finally:
        D.dawn_graph_release(ctx, h)


def test_errors_leave_output_untouched(ctx, upload):
    h, g, src = upload("uniform4096")
    out = np.full(g.n, 123, np.int32)
    for bad in (-1, g.n):
        with pytest.raises(D.DawnError) as ei:
            D.dawn_sssp(ctx, h, bad, out=out)
        assert ei.value.status == D.DAWN_E_INVALID_ARG
    with pytest.raises(D.DawnError) as ei:
        D.dawn_sssp(ctx, 987654, 0, out=out)
    assert ei.value.status == D.DAWN_E_NOT_FOUND
    assert (out == 123).all()


def test_bad_graphs_rejected(ctx):
    cases = [
        (np.array([1, 1], np.int32), np.array([0], np.int32)),          # row_ptr[0] != 0
        (np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32)),    # decreasing
        (np.array([0, 1, 1], np.int32), np.array([5], np.int32)),       # col out of range
        (np.array([0, 1, 2], np.int32), np.array([0, -1], np.int32)),
    ]
    for rp, col in cases:
        with pytest.raises(D.DawnError) as ei:
            D.dawn_graph_upload(ctx, rp, col)
        assert ei.value.status == D.DAWN_E_BAD_GRAPH
    lib = D.load()
    gid = __import__("ctypes").c_int32(-1)
    rp = np.array([0, 1], np.int32)
    col = np.array([0], np.int32)
    st = lib.dawn_graph_upload(ctx, 1, 2, rp.ctypes.data, col.ctypes.data, 0, gid)  # m != row_ptr[n]
    assert st == D.DAWN_E_BAD_GRAPH
    st = lib.dawn_graph_upload(ctx, 0, 0, rp.ctypes.data, col.ctypes.data, 0, gid)
    assert st == D.DAWN_E_INVALID_ARG


def test_repeat_runs_identical(ctx, upload):
    h, g, src = upload("rmat12")
    a, _ = D.dawn_sssp(ctx, h, int(src[0]))
    for _ in range(5):
        b, _ = D.dawn_sssp(ctx, h, int(src[0]))
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["rmat20", "grid2048"])
def test_full_size(ctx, upload, name):
    """Configs 2 and 3 at their stated size: every one of the workload's
    sources (64 on R-MAT 20, 16 on grid 2048^2) in the default driver, each
    row equal to the oracle's, with its level histogram; the other drivers on
    one source."""
    import torch
    h, g, src = upload(name)
    _say(f"[sssp] full size {name} n={g.n} m={g.m}, {src.size} sources")
    rows = torch.empty((src.size, g.n), dtype=torch.int32, device="cuda")
    stats = []
    for i, s in enumerate(src):
        _, st = D.dawn_sssp(ctx, h, int(s), out=rows[i], frontier_cap=8192)
        stats.append(st)
    got = rows.cpu().numpy()
    want = oracle.mssp(g, src, threads=16)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} mismatches, first (row, node) {bad[0]}"
    deg = g.out_degree()
    for r, st in enumerate(stats):
        lv = int(want[r].max()) + 1
        assert st["levels"] == lv
        assert st["source_edges"] == int(deg[want[r] >= 0].sum())
        assert st["frontier_sizes"] == np.bincount(want[r][want[r] >= 0], minlength=lv).tolist()
    _say(f"  levels {min(s['levels'] for s in stats)}..{max(s['levels'] for s in stats)}")
    # the other drivers on one source, and medium push levels on four sources
    saved = D.dawn_get_params(ctx, h)
    try:
        for driver in (1, 2, 4):
            D.dawn_set_params(ctx, h, driver=driver, graph_levels=32)
            got, st = D.dawn_sssp(ctx, h, int(src[0]))
            _check_row(g, src[0], got)
        D.dawn_set_params(ctx, h, driver=3, graph_levels=32, medium_edges=65536)
        for r in range(4):
            got, st = D.dawn_sssp(ctx, h, int(src[r]), frontier_cap=8192)
            assert np.array_equal(got, want[r]), f"medium levels, source {src[r]}"
            assert st["frontier_sizes"] == stats[r]["frontier_sizes"]
    finally:
        D.dawn_set_params(ctx, h, **saved)


def test_small_components_one_workgroup(ctx):
    """Sources in weakly connected components of <= small_n nodes run as one
    workgroup (two launches); results equal the oracle's, and forcing pull or
    small_n = 0 takes the general level loop with the same rows."""
    rng = np.random.default_rng(21)
    edges, base, comps = [], 0, []
    for size in [1, 2, 3, 17, 64, 200, 1000, 2048, 2049, 5000]:
        local = rng.integers(0, size, size=(3 * size, 2)) if size > 1 else np.zeros((0, 2), np.int64)
        chain = [(i, i + 1) for i in range(size - 1)]          # keep it weakly connected
        e = np.concatenate([local, np.array(chain, np.int64).reshape(-1, 2)]) + base
        edges.append(e)
        comps.append((base, size))
        base += size
    g = gg.gen_edges(base, np.concatenate(edges), symmetrize=False, drop_self=False, dedupe=True)
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        D.dawn_set_params(ctx, h, small_n=2048, direction=3)
        for b, size in comps:
            for s in sorted({b, b + size // 2, b + size - 1}):
                got, st = D.dawn_sssp(ctx, h, s, frontier_cap=64)
                _check_row(g, s, got, st)
                if size <= 2048:
                    assert st["launches"] == 2, (size, st["launches"])
                else:
                    assert st["launches"] > 2
        for kw in (dict(small_n=0, direction=3), dict(small_n=2048, direction=2),
                   dict(small_n=2048, direction=1, driver=2)):
            D.dawn_set_params(ctx, h, **kw)
            for b, size in comps[:7]:
                got, st = D.dawn_sssp(ctx, h, b, frontier_cap=64)
                _check_row(g, b, got, st)
    finally:
        D.dawn_graph_release(ctx, h)


def test_level_timing_mode(ctx, upload, restore):
    """Timing mode 1 (driver 2): the level launches alone are timed by events
    attached to their dispatches and by the kernel's own wall-clock stamps;
    the row is unchanged, the clock sum sits inside the event sum."""
    h, g, src = upload("rmat12")
    restore(h, driver=2, timing=1)
    for s in src[:4]:
        got, st = D.dawn_sssp(ctx, h, int(s))
        _check_row(g, s, got, st)
        assert st["launches"] >= st["levels"] - 1
        assert st["kernel_ms"] > 0 and st["kernel_clock_ms"] > 0
        assert st["kernel_clock_ms"] <= st["kernel_ms"] * 1.1 + 0.005, st
    restore(h, driver=3, timing=2)
    _, st = D.dawn_sssp(ctx, h, int(src[0]))
    assert st["kernel_clock_ms"] == 0.0
