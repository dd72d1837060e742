"""Memory-frugal resident form (DAWN_SHARED_CSC): a symmetric graph's CSR
also serves as its in-lists.  Every path (single source in each direction,
batched, APSP, serving) must give the oracle's rows bit for bit, with
4(n+1+m) fewer device bytes; a non-symmetric graph is refused."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["rmat12", "grid128"])
def test_shared_matches_oracle_and_saves_memory(ctx, name):
    g, src = gg.load_config(name)
    h0 = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    h1 = D.dawn_graph_upload(ctx, g.row_ptr, g.col, flags=D.DAWN_SHARED_CSC)
    try:
        b0 = D.dawn_graph_get_info(ctx, h0)["device_bytes"]
        b1 = D.dawn_graph_get_info(ctx, h1)["device_bytes"]
        assert b0 - b1 == 4 * (g.n + 1 + g.m)
        want = oracle.mssp(g, src[:6])
        for direction in (1, 2, 3):
            for driver in (1, 3):
                D.dawn_set_params(ctx, h1, direction=direction, driver=driver)
                for r, s in enumerate(src[:6]):
                    got, _ = D.dawn_sssp(ctx, h1, int(s))
                    assert np.array_equal(got, want[r]), (name, direction, driver, int(s))
        D.dawn_set_params(ctx, h1, direction=3, driver=3)
        got, _ = D.dawn_mssp(ctx, h1, src[:40])
        assert np.array_equal(got, oracle.mssp(g, src[:40]))
        nodes, dist, _ = D.dawn_apsp_wcc(ctx, h1)
        nodes0, dist0, _ = D.dawn_apsp_wcc(ctx, h0)
        assert np.array_equal(nodes, nodes0) and np.array_equal(dist, dist0)
        out = np.empty((5, g.n), np.int32)
        t = D.dawn_serve_submit(ctx, h1, src[:5], out)
        st, _ = D.dawn_serve_wait(ctx, t, 60000)
        assert st == D.DAWN_OK
        assert np.array_equal(out, want[:5])
    finally:
        D.dawn_graph_release(ctx, h0)
        D.dawn_graph_release(ctx, h1)


def test_shared_refuses_directed_graph(ctx):
    g, _ = gg.load_config("uniform4096")         # directed
    with pytest.raises(D.DawnError) as ei:
        D.dawn_graph_upload(ctx, g.row_ptr, g.col, flags=D.DAWN_SHARED_CSC)
    assert ei.value.status == D.DAWN_E_BAD_GRAPH
    # equal in- and out-degrees, not symmetric: a directed 3-cycle
    c = gg.gen_edges(3, [(0, 1), (1, 2), (2, 0)])
    with pytest.raises(D.DawnError) as ei:
        D.dawn_graph_upload(ctx, c.row_ptr, c.col, flags=D.DAWN_SHARED_CSC)
    assert ei.value.status == D.DAWN_E_BAD_GRAPH
    with pytest.raises(D.DawnError) as ei:
        D.dawn_graph_upload(ctx, c.row_ptr, c.col, flags=0x80)
    assert ei.value.status == D.DAWN_E_INVALID_ARG
