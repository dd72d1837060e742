"""Weighted graphs: the (min, +) level loop (dawn_sssp_weighted) against the
weighted oracle (Dijkstra), bit for bit, on tiny random graphs with zero
weights, self-loops and repeated edges, on the test workloads, at R-MAT 20
size, and with unit weights against the unweighted path."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _check(g, w, s, got, st=None):
    want = oracle.wsssp(g, w, int(s))
    assert want.max() < 2**31 - 1
    if not np.array_equal(got.astype(np.int64), want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"source {s}: {bad.size} mismatches, first {bad[:5]}: "
                             f"got {got[bad[:5]]} want {want[bad[:5]]}")
    if st is not None:
        reached = want >= 0
        assert st["reached"] == int(reached.sum())
        assert st["source_edges"] == int(g.out_degree()[reached].sum())


def test_tiny_random_weighted(ctx):
    rng = np.random.default_rng(31)
    for i in range(60):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(0, 4 * n + 1))
        g = gg.gen_edges(n, np.stack([rng.integers(0, n, m), rng.integers(0, n, m)], 1),
                         symmetrize=bool(i % 3 == 0), drop_self=False, dedupe=bool(i % 2))
        w = rng.integers(0, int(rng.choice([1, 5, 100])) + 1, size=g.m).astype(np.int32)
        h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        try:
            D.dawn_graph_set_weights(ctx, h, w)
            for s in range(min(n, 5)):
                got, st = D.dawn_sssp_weighted(ctx, h, s)
                _check(g, w, s, got, st)
        finally:
            D.dawn_graph_release(ctx, h)


@pytest.mark.parametrize("name", ["rmat12", "grid128", "grid128ns", "uniform4096"])
@pytest.mark.parametrize("wrange", [(1, 100), (0, 10)])
def test_workloads_weighted(ctx, name, wrange):
    g, src = gg.load_config(name)
    w = gg.gen_weights(g, wrange[0], wrange[1], seed=9, symmetric=name != "uniform4096")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        D.dawn_graph_set_weights(ctx, h, w)
        hub = int(np.argmax(g.out_degree()))      # its row goes by chunks from round 0
        for s in list(src[:6]) + [hub]:
            got, st = D.dawn_sssp_weighted(ctx, h, int(s))
            _check(g, w, s, got, st)
        _say(f"[weighted] {name} w in {wrange}: rounds {st['levels']}, "
             f"kernel {st['kernel_ms']:.3f} ms")
    finally:
        D.dawn_graph_release(ctx, h)


def test_unit_weights_equal_unweighted(ctx, upload):
    g, src = gg.load_config("rmat12")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        D.dawn_graph_set_weights(ctx, h, np.ones(g.m, np.int32))
        for s in src[:8]:
            got, _ = D.dawn_sssp_weighted(ctx, h, int(s))
            want, _ = D.dawn_sssp(ctx, h, int(s))
            assert np.array_equal(got, want)
    finally:
        D.dawn_graph_release(ctx, h)


@pytest.mark.parametrize("name", ["rmat20", "grid2048"])
def test_full_size_weighted(ctx, upload, name):
    import torch
    h, g, src = upload(name)
    w = gg.gen_weights(g, 1, 100, seed=12, symmetric=True)   # 100 x (n - 1) fits int32
    D.dawn_graph_set_weights(ctx, h, w)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    picks = src[:4]
    rows = []
    for s in picks:
        _, st = D.dawn_sssp_weighted(ctx, h, int(s), out=out)
        torch.cuda.synchronize()
        rows.append(out.cpu().numpy().copy())
        _say(f"[weighted] {name} source {s}: rounds {st['levels']}, kernel {st['kernel_ms']:.2f} ms, "
             f"GTEPS {st['source_edges'] / st['kernel_ms'] / 1e6:.1f}")
    want = oracle.wmssp(g, w, picks, threads=16)
    assert np.array_equal(np.stack(rows).astype(np.int64), want)


def test_weighted_errors(ctx, upload):
    h, g, src = upload("uniform4096")
    g2, _ = gg.load_config("grid128")
    h2 = D.dawn_graph_upload(ctx, g2.row_ptr, g2.col)
    try:
        out = np.full(g2.n, 5, np.int32)
        with pytest.raises(D.DawnError) as ei:             # no weights attached
            D.dawn_sssp_weighted(ctx, h2, 0, out=out)
        assert ei.value.status == D.DAWN_E_INVALID_ARG
        assert (out == 5).all()
        bad = np.ones(g2.m, np.int32)
        bad[7] = -3
        with pytest.raises(D.DawnError) as ei:
            D.dawn_graph_set_weights(ctx, h2, bad)
        assert ei.value.status == D.DAWN_E_INVALID_ARG
        huge = np.full(g2.m, 1 << 20, np.int32)           # 2^20 x (n - 1) overflows int32
        with pytest.raises(D.DawnError) as ei:
            D.dawn_graph_set_weights(ctx, h2, huge)
        assert ei.value.status == D.DAWN_E_INVALID_ARG
        with pytest.raises(ValueError):
            D.dawn_graph_set_weights(ctx, h2, np.ones(g2.m - 1, np.int32))
        # weights replaced by a second call
        D.dawn_graph_set_weights(ctx, h2, np.full(g2.m, 2, np.int32))
        D.dawn_graph_set_weights(ctx, h2, np.full(g2.m, 3, np.int32))
        got, _ = D.dawn_sssp_weighted(ctx, h2, 0)
        want, _ = D.dawn_sssp(ctx, h2, 0)
        assert np.array_equal(got, np.where(want >= 0, 3 * want, -1))
    finally:
        D.dawn_graph_release(ctx, h2)


def test_weighted_device_output(ctx):
    import torch
    g, src = gg.load_config("grid128")
    w = gg.gen_weights(g, 0, 50, seed=2, symmetric=True)
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        D.dawn_graph_set_weights(ctx, h, w)
        out = torch.full((g.n,), 9, dtype=torch.int32, device="cuda")
        D.dawn_sssp_weighted(ctx, h, int(src[0]), out=out)
        torch.cuda.synchronize()
        _check(g, w, src[0], out.cpu().numpy())
    finally:
        D.dawn_graph_release(ctx, h)
