"""The entry point that allocates nothing (dawn_sssp_noalloc): its rows equal
dawn_sssp's, bit for bit, on two calls in a row, the second on a smaller
graph; a graph too large for its static scratch array is refused."""
import sys

import numpy as np
import pytest

import graphgen as gg
from paper_2208_04514_amd import dawn as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def test_no_alloc_matches_sssp(ctx):
    import torch
    runs = []
    for name in ("rmat18", "rmat12", "grid128ns"):      # the second is smaller than the first
        g, src = gg.load_config(name)
        runs.append((name, g, src, D.dawn_graph_upload(ctx, g.row_ptr, g.col)))
    try:
        lib = D.load()
        for name, g, src, h in runs:
            for s in src[:3]:
                want, _ = D.dawn_sssp(ctx, h, int(s))
                out = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
                _say(f"[no_alloc] {name} n={g.n} source {s}")
                st = D.RunStats()
                rc = lib.dawn_sssp_noalloc(ctx, h, int(s), out.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream, st)
                assert rc == D.DAWN_OK, D.dawn_last_error()
                got = out.cpu().numpy()
                assert np.array_equal(got, want), f"{name} source {s}: rows differ"
                assert st.levels == int(want.max()) + 1
        # through the binding, on a side stream
        name, g, src, h = runs[1]
        s2 = torch.cuda.Stream()
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(s2):
            _, st = D.dawn_sssp_noalloc(ctx, h, int(src[5]), out)
        want, _ = D.dawn_sssp(ctx, h, int(src[5]))
        assert np.array_equal(out.cpu().numpy(), want)
    finally:
        for _, _, _, h in runs:
            D.dawn_graph_release(ctx, h)


def test_no_alloc_refuses_large_graph(ctx):
    import torch
    g, src = gg.load_config("rmat20")        # needs far more than the scratch array
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    try:
        out = torch.full((g.n,), 3, dtype=torch.int32, device="cuda")
        with pytest.raises(D.DawnError) as ei:
            D.dawn_sssp_noalloc(ctx, h, int(src[0]), out)
        assert ei.value.status == D.DAWN_E_INVALID_ARG
        assert "no-allocation" in str(ei.value)
        assert bool((out == 3).all())
    finally:
        D.dawn_graph_release(ctx, h)
