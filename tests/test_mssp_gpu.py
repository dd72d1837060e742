"""Batched multi-source parity: every row of dawn_mssp equals the oracle's row for its source."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _check_rows(g, sources, got, stats=None, threads=16):
    want = oracle.mssp(g, sources, threads=threads)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, v = bad[0]
        raise AssertionError(f"{len(bad)} mismatches; first row {r} (source {sources[r]}) node {v}: "
                             f"got {got[r, v]} want {want[r, v]}")
    if stats is not None:
        deg = g.out_degree()
        reached = want >= 0
        assert stats["reached"] == int(reached.sum())
        assert stats["source_edges"] == int((reached.astype(np.int64) @ deg).sum())
        assert stats["levels"] == int(want.max()) + 1
    return want


@pytest.fixture
def params(ctx):
    saved = []

    def _set(h, **kw):
        saved.append((h, D.dawn_get_params(ctx, h)))
        return D.dawn_set_params(ctx, h, **kw)
    yield _set
    for h, p in reversed(saved):
        D.dawn_set_params(ctx, h, **p)


@pytest.mark.parametrize("k", [1, 2, 63, 64, 65, 127, 200])
@pytest.mark.parametrize("direction", [1, 2, 3])
def test_widths_and_directions(ctx, upload, params, k, direction):
    h, g, _ = upload("rmat12")
    params(h, direction=direction)
    src = gg.sample_sources(g.n, k, 1000 + k)
    _say(f"[mssp] rmat12 k={k} direction={direction}")
    got, st = D.dawn_mssp(ctx, h, src)
    _check_rows(g, src, got, st)


@pytest.mark.parametrize("name", ["uniform4096", "grid128", "grid128ns"])
@pytest.mark.parametrize("direction", [1, 2, 3])
def test_workloads(ctx, upload, params, name, direction):
    h, g, src = upload(name)
    params(h, direction=direction)
    srcs = gg.sample_sources(g.n, 300, 77)
    _say(f"[mssp] {name} k=300 direction={direction}")
    got, st = D.dawn_mssp(ctx, h, srcs)
    _check_rows(g, srcs, got, st)


def test_duplicates_and_isolated_sources(ctx, upload, params):
    h, g, src = upload("rmat12")
    deg = g.out_degree()
    zero = np.nonzero(deg == 0)[0][:5].astype(np.int32)
    srcs = np.concatenate([src[:10], src[:10], zero, src[:3]]).astype(np.int32)
    got, st = D.dawn_mssp(ctx, h, srcs)
    want = _check_rows(g, srcs, got, st)
    assert np.array_equal(got[:10], got[10:20])
    for r in range(20, 20 + zero.size):
        assert got[r, srcs[r]] == 0 and (np.delete(got[r], srcs[r]) == -1).all()


def test_permutation_permutes_rows(ctx, upload):
    h, g, src = upload("rmat12")
    srcs = src[:40]
    a, _ = D.dawn_mssp(ctx, h, srcs)
    p = np.random.default_rng(3).permutation(srcs.size)
    b, _ = D.dawn_mssp(ctx, h, srcs[p])
    assert np.array_equal(a[p], b)


def test_many_batches(ctx, upload, params):
    # more sources than one batch holds: batches of 64 lanes, ragged tail
    h, g, _ = upload("uniform4096")
    params(h, batch_lanes=64)
    srcs = gg.sample_sources(g.n, 64 * 3 + 17, 5)
    got, st = D.dawn_mssp(ctx, h, srcs)
    _check_rows(g, srcs, got, st)


def test_level_chunks_deep_then_shallow(ctx, upload):
    """The device-driven loop queues levels in chunks sized from the graph's
    last run: a deep run after a shallow one needs further chunks, a shallow
    run after a deep one leaves queued levels that must do nothing."""
    h, g, _ = upload("grid128ns")
    want0 = oracle.sssp(g, 0)
    far = int(np.argmax(want0))                  # deepest node from corner 0
    mid = int(np.argsort(want0)[g.n // 2])       # a node half-way in
    runs = [np.array([0, far], np.int32), np.array([mid], np.int32),
            np.array([0], np.int32), np.array([mid, far, 0], np.int32)]
    for src in runs:
        _say(f"[mssp] grid128ns chunked levels sources={src.tolist()}")
        got, st = D.dawn_mssp(ctx, h, src)
        _check_rows(g, src, got, st)


@pytest.mark.parametrize("device_out", [False, True])
def test_concurrent_batch_groups(ctx, upload, params, device_out):
    """Ten batches of 64 lanes: groups of four batches run side by side (each
    on its own workspace and stream), the last group holds two, the last
    batch is ragged."""
    h, g, _ = upload("rmat12")
    params(h, batch_lanes=64)
    srcs = gg.sample_sources(g.n, 64 * 9 + 5, 31)
    _say(f"[mssp] rmat12 k={srcs.size} in batches of 64, device_out={device_out}")
    if device_out:
        import torch
        out = torch.full((srcs.size, g.n), 7, dtype=torch.int32, device="cuda")
        _, st = D.dawn_mssp(ctx, h, srcs, out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    else:
        got, st = D.dawn_mssp(ctx, h, srcs)
    _check_rows(g, srcs, got, st)


@pytest.mark.parametrize("k", [4095, 4096, 4097, 5000])
def test_batch_edges(ctx, upload, k):
    h, g, _ = upload("uniform4096")
    srcs = np.concatenate([np.arange(g.n), np.arange(g.n)])[:k].astype(np.int32)
    _say(f"[mssp] uniform4096 k={k}")
    got, st = D.dawn_mssp(ctx, h, srcs)
    _check_rows(g, srcs, got, st)


def test_k_zero_and_errors(ctx, upload):
    h, g, _ = upload("uniform4096")
    out, st = D.dawn_mssp(ctx, h, np.empty(0, np.int32))
    assert out.shape == (0, g.n)
    buf = np.full((2, g.n), 55, np.int32)
    with pytest.raises(D.DawnError) as ei:
        D.dawn_mssp(ctx, h, np.array([0, g.n], np.int32), out=buf)
    assert ei.value.status == D.DAWN_E_INVALID_ARG
    assert (buf == 55).all()


def test_device_output(ctx, upload):
    import torch
    h, g, src = upload("rmat12")
    out = torch.full((src.size, g.n), 9, dtype=torch.int32, device="cuda")
    D.dawn_mssp(ctx, h, src, out=out)
    torch.cuda.synchronize()
    _check_rows(g, src, out.cpu().numpy())


def test_mssp_matches_sssp(ctx, upload):
    h, g, src = upload("grid128")
    got, _ = D.dawn_mssp(ctx, h, src[:8])
    for r, s in enumerate(src[:8]):
        row, _ = D.dawn_sssp(ctx, h, int(s))
        assert np.array_equal(row, got[r])


def test_full_size_rmat18_4096(ctx, upload):
    """The batched workload at full size: R-MAT 18, 4096 sources in one launch,
    every one of the 4096 rows compared with the oracle (16 host threads)."""
    import torch
    h, g, src = upload("rmat18")
    assert src.size == 4096
    out = torch.empty((4096, g.n), dtype=torch.int32, device="cuda")
    _say("[mssp] rmat18 4096 sources")
    _, st = D.dawn_mssp(ctx, h, src, out=out)
    torch.cuda.synchronize()
    _say(f"  levels {st['levels']} push {st['push_levels']} pull {st['pull_levels']} "
         f"kernel {st['kernel_ms']:.2f} ms GTEPS {st['source_edges'] / st['kernel_ms'] / 1e6:.1f}")
    got = out.cpu().numpy()
    del out
    _say("  oracle on all 4096 rows")
    _check_rows(g, src, got, st, threads=16)


def test_host_output_untouched_when_a_later_group_fails(dawn_lib):
    """Host-destination rows are staged on the device and copied out only
    after every batch has finished: a plane allocation refused in the second
    group of side-by-side batches leaves the caller's buffer as it was."""
    import os
    # two directed-both-ways paths: 40 nodes (sources 0..255 sit on it via
    # repeats: runs end before level 29, 6 planes) and 100 nodes (a source at
    # its end needs level 99: a 7th plane, allocated in the second group)
    a, b = 40, 100
    e = [(i, i + 1) for i in range(a - 1)] + [(a + i, a + i + 1) for i in range(b - 1)]
    g = gg.gen_edges(a + b, np.array(e, np.int64), symmetrize=True)
    srcs = np.concatenate([np.resize(np.arange(a), 64 * 4), [a] * 10]).astype(np.int32)
    os.environ["DAWN_FAIL_PLANE_AFTER"] = str(4 * 6)
    try:
        c = D.dawn_create(0, 0)
    finally:
        del os.environ["DAWN_FAIL_PLANE_AFTER"]
    try:
        h = D.dawn_graph_upload(c, g.row_ptr, g.col)
        D.dawn_set_params(c, h, batch_lanes=64)
        out = np.full((srcs.size, g.n), 55, np.int32)
        with pytest.raises(D.DawnError) as ei:
            D.dawn_mssp(c, h, srcs, out=out)
        assert ei.value.status == D.DAWN_E_NO_MEMORY
        assert (out == 55).all(), "a failed call wrote the caller's rows"
        got, st = D.dawn_mssp(c, h, srcs, out=out)      # the injection fired once
        _check_rows(g, srcs, got, st)
    finally:
        D.dawn_destroy(c)


# ------------------------------------------------------- device-ordered runs --

def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, np.int32), device="cuda")


@pytest.mark.parametrize("name", ["rmat12", "grid128ns", "uniform4096"])
def test_device_ordered_rows(ctx, dawn_lib, name):
    """dawn_mssp_device queues everything on the caller's stream: a fresh
    graph queues 8 levels as launches and leaves the rest (grid128ns: about
    250 levels) to the cooperative kernel; the next call queues the depth of
    the finished run.  Rows and status are read after the stream only."""
    import torch
    g, _ = gg.load_config(name)
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)      # fresh: no depth hint yet
    try:
        for k, seed in ((100, 1), (64, 2), (1, 3)):
            srcs = gg.sample_sources(g.n, k, 500 + seed)
            out = torch.full((k, g.n), 9, dtype=torch.int32, device="cuda")
            status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                d_src = _dev(srcs)
                _say(f"[mssp_device] {name} k={k}")
                D.dawn_mssp_device(ctx, h, d_src, out, status)
                res = out.clone()          # ordered after the queued run on s
            s.synchronize()
            assert int(status.item()) == D.DAWN_OK
            _check_rows(g, srcs, res.cpu().numpy())
    finally:
        D.dawn_graph_release(ctx, h)


def test_device_ordered_many_batches_and_streams(ctx, upload, params):
    """Sources beyond one batch run batch after batch on the stream; two
    streams share the graph's workspaces through events."""
    import torch
    h, g, _ = upload("rmat12")
    params(h, batch_lanes=64)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a_src = gg.sample_sources(g.n, 64 * 3 + 5, 41)
    b_src = gg.sample_sources(g.n, 70, 42)
    a_out = torch.empty((a_src.size, g.n), dtype=torch.int32, device="cuda")
    b_out = torch.empty((b_src.size, g.n), dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s1):
        D.dawn_mssp_device(ctx, h, _dev(a_src), a_out)
    with torch.cuda.stream(s2):
        D.dawn_mssp_device(ctx, h, _dev(b_src), b_out)
    torch.cuda.synchronize()
    _check_rows(g, a_src, a_out.cpu().numpy())
    _check_rows(g, b_src, b_out.cpu().numpy())
    # the synchronous call after device-ordered ones on the same workspaces
    got, st = D.dawn_mssp(ctx, h, b_src)
    _check_rows(g, b_src, got, st)


def test_device_ordered_errors(ctx, upload):
    """An invalid source is found on the device: status INVALID_ARG and no row
    written; host-side errors return at once; k == 0 writes only the status."""
    import torch
    h, g, src = upload("rmat12")
    srcs = src[:10].copy()
    srcs[7] = g.n
    out = torch.full((10, g.n), 5, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    D.dawn_mssp_device(ctx, h, _dev(srcs), out, status)
    torch.cuda.synchronize()
    assert int(status.item()) == D.DAWN_E_INVALID_ARG
    assert bool((out == 5).all())
    # the workspace is usable afterwards
    D.dawn_mssp_device(ctx, h, _dev(src[:10]), out, status)
    torch.cuda.synchronize()
    assert int(status.item()) == D.DAWN_OK
    _check_rows(g, src[:10], out.cpu().numpy())
    empty = torch.empty((0, g.n), dtype=torch.int32, device="cuda")
    D.dawn_mssp_device(ctx, h, _dev(np.empty(0, np.int32)), empty, status)
    torch.cuda.synchronize()
    assert int(status.item()) == D.DAWN_OK
    lib = D.load()
    host = np.zeros((10, g.n), np.int32)
    d_src = _dev(src[:10])
    st = lib.dawn_mssp_device(ctx, h, d_src.data_ptr(), 10, host.ctypes.data, None, None)
    assert st == D.DAWN_E_INVALID_ARG and "device memory" in D.dawn_last_error()
    small = torch.empty((9, g.n), dtype=torch.int32, device="cuda")
    big_k = 1 << 20
    st = lib.dawn_mssp_device(ctx, h, d_src.data_ptr(), big_k, small.data_ptr(), None, None)
    assert st == D.DAWN_E_INVALID_ARG
    st = lib.dawn_mssp_device(ctx, 987654, d_src.data_ptr(), 10, out.data_ptr(), None, None)
    assert st == D.DAWN_E_NOT_FOUND
