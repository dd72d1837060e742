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
                dict(timing=1, driver=3)):
        with pytest.raises(D.DawnError) as ei:
            D.dawn_set_params(ctx, h, **bad)
        assert ei.value.status == D.DAWN_E_INVALID_ARG
    assert D.dawn_get_params(ctx, h) == before
