"""The host CPU DAWN (libdawn_host, the SOVM level loop on CPU threads)
against the CPU oracle, bit for bit, at several thread counts.  CPU only."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from conftest import load_golden
from paper_2208_04514_amd import dawn_host as H


@pytest.fixture(scope="module", autouse=True)
def built():
    from paper_2208_04514_amd.host import build
    build.build()
    H.load()


@pytest.mark.parametrize("name", ["uniform4096", "rmat12", "grid128", "grid128ns"])
@pytest.mark.parametrize("threads", [1, 2, 3, 8])
def test_sssp_matches_oracle(name, threads):
    g, src = gg.load_config(name)
    hg = H.HostGraph(g.row_ptr, g.col)
    deg = g.out_degree()
    for s in src[:4]:
        got, st = H.dawn_host_sssp(hg, int(s), threads)
        want = oracle.sssp(g, int(s))
        assert np.array_equal(got, want), (name, threads, int(s))
        assert st["levels"] == int(want.max()) + 1
        assert st["reached"] == int((want >= 0).sum())
        assert st["source_edges"] == int(deg[want >= 0].sum())


@pytest.mark.parametrize("threads", [1, 4])
def test_mssp_matches_oracle(threads):
    g, src = gg.load_config("rmat12")
    hg = H.HostGraph(g.row_ptr, g.col)
    srcs = np.concatenate([src[:20], src[:3]])          # duplicates give identical rows
    got, st = H.dawn_host_mssp(hg, srcs, threads)
    want = oracle.mssp(g, srcs)
    assert np.array_equal(got, want)
    assert st["reached"] == int((want >= 0).sum())
    got0, _ = H.dawn_host_mssp(hg, np.zeros(0, np.int32), threads)
    assert got0.shape == (0, g.n)


def test_tiny_random_graphs():
    rng = np.random.default_rng(11)
    for i in range(60):
        n = int(rng.integers(1, 120))
        m = int(rng.integers(0, 4 * n))
        e = rng.integers(0, n, size=(m, 2))
        g = gg.gen_edges(n, e, symmetrize=bool(i % 2), drop_self=False, dedupe=bool(i % 3))
        hg = H.HostGraph(g.row_ptr, g.col)
        for s in sorted(set(rng.integers(0, n, size=3).tolist())):
            for t in (1, 3):
                got, _ = H.dawn_host_sssp(hg, s, t)
                assert np.array_equal(got, oracle.sssp(g, s))


@pytest.mark.parametrize("name", ["hand_directed10.txt", "petersen.txt"])
def test_golden(name):
    n, edges, rows = load_golden(name)
    g = gg.gen_edges(n, edges, drop_self=False, dedupe=False)
    hg = H.HostGraph(g.row_ptr, g.col)
    for s, want in rows.items():
        for t in (1, 2):
            got, _ = H.dawn_host_sssp(hg, s, t)
            assert np.array_equal(got, want)


def test_edge_cases_and_errors():
    g = gg.gen_edges(1, np.zeros((0, 2), np.int64))
    hg = H.HostGraph(g.row_ptr, g.col)
    got, st = H.dawn_host_sssp(hg, 0, 4)
    assert got.tolist() == [0] and st["levels"] == 1
    g = gg.gen_edges(5, [(0, 1), (1, 2)])
    hg = H.HostGraph(g.row_ptr, g.col)
    got, _ = H.dawn_host_sssp(hg, 3, 2)               # out-degree-0 source
    assert got.tolist() == [-1, -1, -1, 0, -1]
    out = np.full(5, 9, np.int32)
    for bad in (-1, 5):
        with pytest.raises(H.DawnHostError) as ei:
            H.dawn_host_sssp(hg, bad, 1, out=out)
        assert ei.value.status == -1
    with pytest.raises(H.DawnHostError):
        H.dawn_host_sssp(hg, 0, 0, out=out)
    assert (out == 9).all()
    with pytest.raises(H.DawnHostError) as ei:
        H.HostGraph(np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32))
    assert ei.value.status == -2
    with pytest.raises(H.DawnHostError) as ei:
        H.HostGraph(np.array([0, 1], np.int32), np.array([3], np.int32))
    assert ei.value.status == -2


def test_header_symbols_exported():
    import re
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "include", "dawn_host.h")).read()
    names = set(re.findall(r"\b(dawn_host_\w+)\s*\(", text))
    lib = H.load()
    for nm in names:
        assert hasattr(lib, nm), nm
    assert {"dawn_host_sssp", "dawn_host_mssp", "dawn_host_graph_create"} <= names
