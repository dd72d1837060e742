"""Failure handling forced from the host: injected allocation failure, a tiny
budget, and the level-loop's error paths.  No kernel faults on purpose."""
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


def test_injected_allocation_failure(dawn_lib):
    g, src = gg.load_config("uniform4096")
    os.environ["DAWN_FAIL_ALLOC_AFTER"] = "0"
    try:
        ctx = D.dawn_create(0, 0)
    finally:
        del os.environ["DAWN_FAIL_ALLOC_AFTER"]
    try:
        with pytest.raises(D.DawnError) as ei:
            D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        assert ei.value.status == D.DAWN_E_NO_MEMORY
        used, _ = D.dawn_memory(ctx)
        assert used == 0, "a failed upload must not leak device memory"
        h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)     # the next allocation succeeds
        got, _ = D.dawn_sssp(ctx, h, int(src[0]))
        assert np.array_equal(got, oracle.sssp(g, int(src[0])))
    finally:
        D.dawn_destroy(ctx)


def test_budget_too_small_for_workspace(dawn_lib):
    g, src = gg.load_config("rmat12")
    ctx = D.dawn_create(0, int(1.8 * (1 << 20)))   # graph + one source fit, 64 rows do not
    try:
        h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        out = np.full((64, g.n), 5, np.int32)
        with pytest.raises(D.DawnError) as ei:
            D.dawn_mssp(ctx, h, src, out=out)
        assert ei.value.status == D.DAWN_E_NO_MEMORY
        assert (out == 5).all()
        got, _ = D.dawn_sssp(ctx, h, int(src[0]))     # a single source still fits
        assert np.array_equal(got, oracle.sssp(g, int(src[0])))
    finally:
        D.dawn_destroy(ctx)


def test_release_while_idle_and_reuse(ctx, upload):
    g, src = gg.load_config("grid128")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    D.dawn_sssp(ctx, h, int(src[0]))
    D.dawn_graph_release(ctx, h)
    with pytest.raises(D.DawnError) as ei:
        D.dawn_sssp(ctx, h, int(src[0]))
    assert ei.value.status == D.DAWN_E_NOT_FOUND
    with pytest.raises(D.DawnError) as ei:
        D.dawn_graph_release(ctx, h)
    assert ei.value.status == D.DAWN_E_NOT_FOUND
