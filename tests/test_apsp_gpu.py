"""APSP over the largest weakly connected component (dawn_apsp_wcc)."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _check(ctx, h, g, threads=16, symmetric=True):
    nodes, dist, st = D.dawn_apsp_wcc(ctx, h)
    want_nodes = oracle.largest_wcc(g)
    assert np.array_equal(nodes, want_nodes)
    S = nodes.size
    assert dist.shape == (S, S)
    full = oracle.mssp(g, nodes, threads=threads)
    want = full[:, nodes]
    # every finite distance from a WCC node stays inside the WCC
    assert ((full >= 0).sum(1) == (want >= 0).sum(1)).all()
    if not np.array_equal(dist, want):
        bad = np.argwhere(dist != want)
        i, j = bad[0]
        raise AssertionError(f"{len(bad)} mismatches; first ({i},{j}): got {dist[i, j]} want {want[i, j]}")
    assert (np.diag(dist) == 0).all()
    if symmetric:
        # a symmetric graph's WCC is connected and distances are symmetric
        assert (dist >= 0).all()
        assert np.array_equal(dist, dist.T)
    return nodes, dist, st


def test_rmat12(ctx, upload):
    h, g, _ = upload("rmat12")
    _check(ctx, h, g)


def test_directed_uniform(ctx, upload):
    h, g, _ = upload("uniform4096")
    _check(ctx, h, g, symmetric=False)


def test_query_only_and_device_out(ctx, upload):
    import torch
    h, g, _ = upload("grid128")
    nodes, none, _ = D.dawn_apsp_wcc(ctx, h, query_only=True)
    assert none is None and np.array_equal(nodes, oracle.largest_wcc(g))
    out = torch.empty((nodes.size, nodes.size), dtype=torch.int32, device="cuda")
    D.dawn_apsp_wcc(ctx, h, out=out)
    torch.cuda.synchronize()
    want = oracle.mssp(g, nodes, threads=16)[:, nodes]
    assert np.array_equal(out.cpu().numpy(), want)
    info = D.dawn_graph_get_info(ctx, h)
    assert info["s_wcc"] == nodes.size


def test_tie_break_and_tiny(ctx):
    # two components of three nodes; the one holding node 0 wins
    g = gg.gen_edges(7, [(1, 0), (1, 2), (4, 3), (5, 4)])
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        nodes, dist, _ = D.dawn_apsp_wcc(ctx, h)
        assert nodes.tolist() == [0, 1, 2]
        assert dist.tolist() == [[0, -1, -1], [1, 0, 1], [-1, -1, 0]]
    finally:
        D.dawn_graph_release(ctx, h)
    g = gg.gen_edges(1, np.zeros((0, 2), np.int64))
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        nodes, dist, _ = D.dawn_apsp_wcc(ctx, h)
        assert nodes.tolist() == [0] and dist.tolist() == [[0]]
    finally:
        D.dawn_graph_release(ctx, h)


def test_full_size_rmat14(ctx, upload):
    """R-MAT 14: the whole largest WCC (~12.5 K sources, 4 batches of 4096)."""
    h, g, _ = upload("rmat14")
    _say("[apsp] rmat14")
    nodes, dist, st = _check(ctx, h, g, threads=16)
    _say(f"  S_wcc {nodes.size} levels {st['levels']} kernel {st['kernel_ms']:.1f} ms "
         f"GTEPS {st['source_edges'] / st['kernel_ms'] / 1e6:.1f}")
