"""Autotuner: the chosen settings are valid and keep every result bit-exact."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["rmat12", "grid128"])
def test_autotune_keeps_parity(ctx, name):
    g, src = gg.load_config(name)
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        tune_src = gg.sample_sources(g.meta["wcc_nodes"], 64, 4242)
        best = D.dawn_autotune(ctx, h, tune_src, what=3)
        assert best == D.dawn_get_params(ctx, h)
        want = oracle.mssp(g, src[:16])
        for r, s in enumerate(src[:16]):
            got, _ = D.dawn_sssp(ctx, h, int(s))
            assert np.array_equal(got, want[r])
        got, _ = D.dawn_mssp(ctx, h, src[:16])
        assert np.array_equal(got, want)
    finally:
        D.dawn_graph_release(ctx, h)


def test_autotune_bad_args(ctx, upload):
    h, g, src = upload("uniform4096")
    with pytest.raises(D.DawnError) as ei:
        D.dawn_autotune(ctx, h, np.empty(0, np.int32))
    assert ei.value.status == D.DAWN_E_INVALID_ARG
    with pytest.raises(D.DawnError) as ei:
        D.dawn_autotune(ctx, h, src[:2], what=4)
    assert ei.value.status == D.DAWN_E_INVALID_ARG


def test_set_params_validation(ctx, upload):
    h, g, src = upload("uniform4096")
    before = D.dawn_get_params(ctx, h)
    for bad in (dict(driver=9), dict(block=128), dict(batch_lanes=100), dict(big_degree=10),
                dict(timing=1, driver=3), dict(batch_big_degree=32), dict(batch_wide_scan=600),
                dict(batch_sparse_words=5), dict(small_frontier_edges=-3),
                dict(medium_edges=-1), dict(medium_groups=1), dict(medium_groups=300)):
        with pytest.raises(D.DawnError) as ei:
            D.dawn_set_params(ctx, h, **bad)
        assert ei.value.status == D.DAWN_E_INVALID_ARG
    assert D.dawn_get_params(ctx, h) == before


@pytest.mark.parametrize("name", ["rmat12", "grid128ns"])
@pytest.mark.parametrize("k", [100, 2000])
def test_batched_knob_candidates_bit_exact(ctx, upload, name, k):
    """Every candidate value the autotuner tries for the batched knobs gives
    the oracle's rows (narrow rows, k = 100, and wide ones, k = 2000)."""
    h, g, _ = upload(name)
    srcs = gg.sample_sources(g.n, k, 77 + k)
    want = oracle.mssp(g, srcs, threads=16)
    saved = D.dawn_get_params(ctx, h)
    try:
        for knob, vals in (("batch_alpha", (1e-4, 0.25, 1, 4, 16, 64, 1e6)),
                           ("batch_big_degree", (64, 128, 256, 1024)),
                           ("batch_wide_scan", (16, 32, 48, 96, 192)),
                           ("batch_sparse_words", (1, 2, 4))):
            for v in vals:
                D.dawn_set_params(ctx, h, **{knob: v})
                got, _ = D.dawn_mssp(ctx, h, srcs)
                assert np.array_equal(got, want), f"{name} k={k} {knob}={v}"
            D.dawn_set_params(ctx, h, **saved)
    finally:
        D.dawn_set_params(ctx, h, **saved)


@pytest.mark.parametrize("name", ["rmat12", "grid128"])
def test_plain_knob_candidates_bit_exact(ctx, upload, name):
    """Every value the autotuner tries for the single-source level-loop knobs
    gives the oracle's rows."""
    h, g, src = upload(name)
    want = oracle.mssp(g, src[:4])
    saved = D.dawn_get_params(ctx, h)
    try:
        for knob, vals in (("small_frontier_edges", (-1, 128, 256, 512, 1024)),
                           ("big_degree", (128, 256, 512, 1024, 2048, 8192)),
                           ("medium_edges", (0, 4096, 16384, 65536))):
            for v in vals:
                D.dawn_set_params(ctx, h, **{knob: v})
                for r, s in enumerate(src[:4]):
                    got, _ = D.dawn_sssp(ctx, h, int(s))
                    assert np.array_equal(got, want[r]), f"{name} {knob}={v} source {s}"
            D.dawn_set_params(ctx, h, **saved)
        for v in (8, 16, 32, 64):
            D.dawn_set_params(ctx, h, medium_edges=65536, medium_groups=v)
            for r, s in enumerate(src[:4]):
                got, _ = D.dawn_sssp(ctx, h, int(s))
                assert np.array_equal(got, want[r]), f"{name} medium_groups={v} source {s}"
    finally:
        D.dawn_set_params(ctx, h, **saved)


def test_tuned_settings_round_trip_the_cache(ctx, tmp_path):
    """Settings found by dawn_autotune go to the on-disk cache under (arch,
    graph signature, batch width) and come back to give the same rows."""
    from paper_2208_04514_amd import tune_cache as T
    g, src = gg.load_config("rmat12")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    path = str(tmp_path / "tuned.json")
    try:
        best = D.dawn_autotune(ctx, h, src[:64], what=2)
        arch, sig = T.device_arch(0), T.graph_signature(g.row_ptr, g.col)
        assert arch.startswith("gfx")
        T.store(arch, sig, 64, best, path)
        h2 = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        try:
            loaded = T.lookup(arch, sig, 64, path)
            D.dawn_set_params(ctx, h2, **loaded)
            assert D.dawn_get_params(ctx, h2) == best
            got, _ = D.dawn_mssp(ctx, h2, src[:64])
            assert np.array_equal(got, oracle.mssp(g, src[:64]))
        finally:
            D.dawn_graph_release(ctx, h2)
    finally:
        D.dawn_graph_release(ctx, h)
