"""Benchmark: GTEPS of DAWN's level loop on one MI355X.

Headline (``value``): plain per-source SSSP on R-MAT scale 20 (1,048,576 nodes,
edge factor 16, a/b/c/d = .57/.19/.19/.05, symmetrised, de-duplicated), 64
sources from the largest WCC, run one source at a time through ``dawn_sssp``
with device-resident output.  One step = the 64 sources.  GTEPS counts, per
source, the out-degrees of every reached node (the SOVM cost E_wcc(s) of
Section 4), summed over sources, per second.

Also reported on the same JSON line: the batched form (R-MAT scale 18, 4096
sources in one ``dawn_mssp`` launch) next to the same 4096 sources run plain,
APSP over the largest WCC of R-MAT scale 14, the damaged 2048^2 grid under
each level-loop driver, the serving loop (three resident graphs, Poisson
arrivals, p50/p99 latency), the roofline of the level-step kernel, and the
CPU oracle timed on the host cores.

Inputs are seeded synthetic graphs standing in for the paper's
SuiteSparse/Gunrock graphs, which are not available here.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# The knobs of the plain level loop that the bench takes from the tuning
# cache (paper_2208_04514_amd/tuned_params.json, written by dawn_autotune on
# 32 other sources of the same graph; --autotune searches again live).
PLAIN_KNOB_NAMES = ("driver", "graph_levels", "big_degree", "alpha", "beta", "block",
                    "blocks_per_cu", "pull_lane_edges", "small_frontier_edges", "medium_edges",
                    "medium_groups")
BATCH_KNOB_NAMES = ("batch_alpha", "batch_big_degree", "batch_wide_scan", "batch_sparse_words")

# Sources that define the level-step kernel: the HBM counter record under
# profiles/ holds their digest and is used only while it matches.
KERNEL_SOURCES = ["paper_2208_04514_amd/csrc/sssp.hip", "paper_2208_04514_amd/csrc/device_util.hpp",
                  "paper_2208_04514_amd/csrc/internal.hpp", "paper_2208_04514_amd/build.py"]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "sssp_level_rmat20_hbm_counters.md")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def host_cores() -> int:
    """CPUs this process may run on (its affinity set), at most the 16 that
    one GPU's share of the box provides."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def kernel_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record():
    """The committed FETCH_SIZE/WRITE_SIZE record of the level kernel, or None."""
    try:
        with open(TRAFFIC_RECORD) as f:
            for line in f:
                if line.startswith("traffic-record:"):
                    return json.loads(line.split(":", 1)[1])
    except (OSError, ValueError):
        pass
    return None


def plain_alg_bytes(g, dist_rows, levels) -> float:
    """Bytes the push-only level loop must move per the method (all sources summed).

    4 B per out-edge of every reached node (col), 16 B per reached node
    (row_ptr pair, dist write, queue write and read) and one visited-bitmap
    pass (n/8 B) per level; the -1 fill of dist belongs to the init kernel.
    """
    deg = g.out_degree()
    total = 0.0
    for d, lv in zip(dist_rows, levels):
        reached = d >= 0
        total += 4.0 * deg[reached].sum() + 16.0 * reached.sum() + lv * g.n / 8.0
    return total


def run_plain(D, ctx, h, src, out, steps, warmup):
    """Time `steps` passes over the sources; returns (source edges, seconds,
    summed kernel ms, levels of the last pass, per-call wall ms)."""
    import torch
    for _ in range(warmup):
        for i, s in enumerate(src):
            D.dawn_sssp(ctx, h, int(s), out=out[i])
    torch.cuda.synchronize()
    se, ks, levels, calls = 0, 0.0, [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        levels = []
        for i, s in enumerate(src):
            c0 = time.perf_counter()
            _, st = D.dawn_sssp(ctx, h, int(s), out=out[i])
            calls.append((time.perf_counter() - c0) * 1e3)
            se += st["source_edges"]
            ks += st["kernel_ms"]
            levels.append(st["levels"])
    torch.cuda.synchronize()
    return se, time.perf_counter() - t0, ks, levels, np.array(calls)


def level_kernel_timing(D, ctx, h, src, out):
    """Per-launch time of the level-step kernel, measured with HIP events
    attached to each launch on the stream it runs on (library timing mode 1,
    which issues the same level launches one per host check; the events take
    the dispatch's own begin and end timestamps).  The same pass also
    sums each launch's own duration by the GPU's wall clock (first workgroup
    start to last workgroup end, no dispatch gap).
    Returns (total event ms, launches, levels per source, total clock ms)."""
    p = D.dawn_get_params(ctx, h)
    D.dawn_set_params(ctx, h, driver=2, timing=1)
    ms, launches, levels, clk = 0.0, 0, [], 0.0
    try:
        for i, s in enumerate(src):
            _, st = D.dawn_sssp(ctx, h, int(s), out=out[i])
            ms += st["kernel_ms"]
            clk += st["kernel_clock_ms"]
            launches += st["launches"]
            levels.append(st["levels"])
    finally:
        D.dawn_set_params(ctx, h, **p)
    return ms, launches, levels, clk


def roofline_entry(g, dist_rows, lk_ms, lk_launches, lk_levels, knobs, lk_clock_ms=0.0):
    alg = plain_alg_bytes(g, dist_rows, lk_levels)
    achieved = alg / (lk_ms / 1e3) / 1e9
    achieved_clk = alg / (lk_clock_ms / 1e3) / 1e9 if lk_clock_ms > 0 else None
    rec = traffic_record()
    traffic, note = None, "no counter record"
    if rec is not None:
        if rec.get("digest") != kernel_digest():
            note = "level kernel changed since the counters were taken"
        elif rec.get("params") != knobs:
            note = "knobs differ from the counter run"
        else:
            traffic = rec["bytes_per_launch"]
            note = rec.get("source", "")
    # the measured traffic (counter bytes per launch, from the committed
    # record) over the same launch time: the achieved HBM fraction
    traffic_gbs = traffic / (lk_ms / lk_launches / 1e3) / 1e9 if traffic else None
    return {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
        "kernel": "sssp_level", "launches": lk_launches,
        "avg_launch_us": round(lk_ms / lk_launches * 1e3, 3),
        # the launches' own time (GPU wall clock in the kernel; what a
        # profiler's kernel trace reports) and the fraction it gives
        "avg_kernel_clock_us": round(lk_clock_ms / lk_launches * 1e3, 3) if lk_clock_ms else None,
        "achieved_kernel_clock": round(achieved_clk, 2) if achieved_clk else None,
        "frac_kernel_clock": round(achieved_clk / HBM_PEAK_GBS, 5) if achieved_clk else None,
        "alg_bytes_per_launch": round(alg / lk_launches, 1),
        "achieved_traffic": round(traffic_gbs, 2) if traffic_gbs else None,
        "frac_traffic": round(traffic_gbs / HBM_PEAK_GBS, 5) if traffic_gbs else None,
        "traffic_note": note,
    }


def component_edge_sums(g):
    """Per node: sum of out-degrees over its weakly connected component.

    For a symmetric graph this is E_reach of every source in the component
    (reachability = the component), the GTEPS numerator of a served source."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    a = csr_matrix((np.ones(g.m, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    _, lab = connected_components(a, directed=True, connection="weak")
    sums = np.bincount(lab, weights=g.out_degree().astype(np.float64))
    return sums[lab].astype(np.int64)


def batched_only(D, ctx):
    """R-MAT 18, the 4096 bench sources in one dawn_mssp call, three times with
    the cached tuned knobs: the batched kernels alone, for a profiler."""
    import torch
    import graphgen as gg
    g, src = gg.load_config("rmat18")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    cached_knobs(D, ctx, h, g, 4096, PLAIN_KNOB_NAMES + BATCH_KNOB_NAMES, 3, 9002, 4096, False, None)
    out = torch.empty((src.size, g.n), dtype=torch.int32, device="cuda")
    runs = []
    for _ in range(3):
        _, st = D.dawn_mssp(ctx, h, src, out=out)
        runs.append(round(st["kernel_ms"], 3))
    torch.cuda.synchronize()
    print(json.dumps({"batched_only": {"workload": "rmat18_ef16_sym_4096src_one_launch",
                                       "kernel_ms": runs, "levels": st["levels"],
                                       "push_levels": st["push_levels"],
                                       "pull_levels": st["pull_levels"]}}), flush=True)


def cached_knobs(D, ctx, h, g, width, names, what, seed, k_tune, live, tune_file):
    """Knob settings for graph h from the tuning cache, or from a live
    dawn_autotune run (on k_tune other sources of the graph) that is then
    recorded.  Returns (knobs, where they came from, seconds spent tuning)."""
    import graphgen as gg
    from paper_2208_04514_amd import tune_cache as T
    arch, sig = T.device_arch(0), T.graph_signature(g.row_ptr, g.col)
    cached = None if live else T.lookup(arch, sig, width, tune_file)
    if cached is not None and all(n in cached for n in names):
        knobs = {n: cached[n] for n in names}
        D.dawn_set_params(ctx, h, **knobs)
        return knobs, f"tuning cache {os.path.basename(tune_file or T.DEFAULT_PATH)}", 0.0
    t0 = time.perf_counter()
    tuned = D.dawn_autotune(ctx, h, gg.sample_sources(g.meta["wcc_nodes"], k_tune, seed), what=what)
    tune_s = time.perf_counter() - t0
    T.store(arch, sig, width, tuned, tune_file, note=f"{g.name}: dawn_autotune what={what}")
    return {n: tuned[n] for n in names}, "autotune (live)", tune_s


def batched_roofline(g, k, st):
    words = (k + 63) // 64
    alg = st["levels"] * (4.0 * g.n + 4.0 * g.m + 24.0 * words * g.n) + 4.0 * k * g.n
    achieved = alg / (st["kernel_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "alg_bytes": round(alg), "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "kernels": "batch_seed, batch_control, batch_push, batch_pull, batch_merge, "
                       "batch_emit (per-kernel bytes: profiles/batch_rmat18_4096_kernels_hbm.md)"}


def batched_bench(D, ctx, live=False, tune_file=None):
    """R-MAT 18, 4096 sources in one dawn_mssp launch, and the same sources
    one at a time through dawn_sssp."""
    import torch
    import graphgen as gg
    g, src = gg.load_config("rmat18")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    out = torch.empty((src.size, g.n), dtype=torch.int32, device="cuda")
    tuned, tuned_from, tune_s = cached_knobs(D, ctx, h, g, 4096,
                                             PLAIN_KNOB_NAMES + BATCH_KNOB_NAMES, 3, 9002, 4096,
                                             live, tune_file)
    D.dawn_mssp(ctx, h, src, out=out)
    torch.cuda.synchronize()
    times, st_b = [], None
    for _ in range(3):
        t0 = time.perf_counter()
        _, st_b = D.dawn_mssp(ctx, h, src, out=out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    tb = float(np.median(times))
    kept = out[:256].cpu().numpy()      # rows of the timed call, for the oracle leg
    del out
    row = torch.empty(g.n, dtype=torch.int32, device="cuda")
    t0 = time.perf_counter()
    sep = 0
    for s in src:
        _, st = D.dawn_sssp(ctx, h, int(s), out=row)
        sep += st["source_edges"]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    D.dawn_graph_release(ctx, h)
    return {
        "workload": "rmat18_ef16_sym_4096src_one_launch", "n": g.n, "m": g.m,
        "gteps": round(st_b["source_edges"] / tb / 1e9, 2),
        "gteps_device": round(st_b["source_edges"] / st_b["kernel_ms"] / 1e6, 2),
        # the whole call against HBM: per level 4n + 4m (CSC/CSR) + 24 W n
        # (row reads and writes of vis and the next frontier), once 4 k n (output)
        "roofline": batched_roofline(g, src.size, st_b),
        "ms": round(tb * 1e3, 3), "kernel_ms": round(st_b["kernel_ms"], 3),
        "levels": st_b["levels"], "push_levels": st_b["push_levels"],
        "pull_levels": st_b["pull_levels"],
        "plain_same_sources_gteps": round(sep / tp / 1e9, 2),
        "plain_same_sources_ms": round(tp * 1e3, 1),
        "speedup_vs_plain": round(tp / tb, 2),
        "tuned": tuned, "tuned_from": tuned_from,
        "autotune_s": round(tune_s, 2),
        "_kept": (g, src[:256], kept),
    }


def apsp_bench(D, ctx):
    """APSP over the largest WCC of R-MAT 14 (dawn_apsp_wcc, device output)."""
    import torch
    import graphgen as gg
    g, _ = gg.load_config("rmat14")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    nodes, _, _ = D.dawn_apsp_wcc(ctx, h, query_only=True)
    s = nodes.size
    out = torch.empty((s, s), dtype=torch.int32, device="cuda")
    D.dawn_apsp_wcc(ctx, h, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, st = D.dawn_apsp_wcc(ctx, h, out=out)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    D.dawn_graph_release(ctx, h)
    return {"workload": "rmat14_ef16_sym_apsp_largest_wcc", "s_wcc": int(s),
            "ms": round(t * 1e3, 3), "kernel_ms": round(st["kernel_ms"], 3),
            "gteps": round(st["source_edges"] / t / 1e9, 2), "levels": st["levels"]}


def uniform_bench(D, ctx, reps=20):
    """The small CPU-checkable case: directed uniform n = 4096, m = 32,768, its
    8 sources one at a time through dawn_sssp (device output), with the
    per-level cost; latency-bound by construction (a few levels of a few
    hundred nodes)."""
    import torch
    import graphgen as gg
    g, src = gg.load_config("uniform4096")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    out = torch.empty((src.size, g.n), dtype=torch.int32, device="cuda")
    for i, s in enumerate(src):
        D.dawn_sssp(ctx, h, int(s), out=out[i])
    torch.cuda.synchronize()
    calls, se, ks, lv = [], 0, 0.0, 0
    t0 = time.perf_counter()
    for _ in range(reps):
        for i, s in enumerate(src):
            c0 = time.perf_counter()
            _, st = D.dawn_sssp(ctx, h, int(s), out=out[i])
            calls.append((time.perf_counter() - c0) * 1e6)
            se += st["source_edges"]
            ks += st["kernel_ms"]
            lv += st["levels"]
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    rows = out.cpu().numpy()
    D.dawn_graph_release(ctx, h)
    return rows, {"workload": "uniform4096_m32768_directed_8src_plain_sssp", "n": g.n, "m": g.m,
            "sources": int(src.size), "gteps": round(se / t / 1e9, 4),
            "gteps_device": round(se / ks / 1e6, 4),
            "us_per_source_p50": round(float(np.percentile(calls, 50)), 1),
            "us_per_source_p99": round(float(np.percentile(calls, 99)), 1),
            "us_per_level": round(t / lv * 1e6, 2), "levels_per_source": round(lv / reps / src.size, 2)}


def weighted_bench(D, ctx):
    """Weighted graphs (the (min, +) level loop): R-MAT 20 and grid 2048^2
    with seeded integer weights 1..100, equal in both directions; sources of
    the plain workloads, one at a time, device output."""
    import torch
    import graphgen as gg
    res = {}
    for name, k in (("rmat20", 8), ("grid2048", 2)):
        g, src = gg.load_config(name)
        w = gg.gen_weights(g, 1, 100, seed=12, symmetric=True)
        h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        D.dawn_graph_set_weights(ctx, h, w)
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        D.dawn_sssp_weighted(ctx, h, int(src[0]), out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        se, ks, rounds = 0, 0.0, []
        for s in src[:k]:
            _, st = D.dawn_sssp_weighted(ctx, h, int(s), out=out)
            se += st["source_edges"]
            ks += st["kernel_ms"]
            rounds.append(st["levels"])
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[name] = {"sources": k, "weights": "uniform 1..100, symmetric",
                     "ms_per_source": round(t / k * 1e3, 3), "gteps": round(se / t / 1e9, 3),
                     "gteps_device": round(se / ks / 1e6, 3), "rounds": rounds}
        D.dawn_graph_release(ctx, h)
    return res


def small_component_bench(D, ctx):
    """Sources in small components (512 components of 16..2048 nodes): every
    one on one workgroup (small_n = 2048), those in components of at most 512
    nodes (the default), and none (small_n = 0, the general level loop)."""
    import torch
    import graphgen as gg
    g, src = gg.load_config("islands")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    res = {"workload": f"islands: 512 symmetric components of 16..2048 nodes (n={g.n}, m={g.m}), "
                       f"{src.size} sources"}
    rows = {}
    for label, sn in (("one_workgroup", 2048), ("default_512", 512), ("level_loop", 0)):
        D.dawn_set_params(ctx, h, small_n=sn)
        D.dawn_sssp(ctx, h, int(src[0]), out=out)
        t0 = time.perf_counter()
        se = 0
        for s in src:
            _, st = D.dawn_sssp(ctx, h, int(s), out=out)
            se += st["source_edges"]
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[label] = {"us_per_source": round(t / src.size * 1e6, 1), "gteps": round(se / t / 1e9, 4)}
        rows[label] = out.cpu().numpy().copy()
    res["same_last_row"] = bool(np.array_equal(rows["one_workgroup"], rows["level_loop"])
                                and np.array_equal(rows["default_512"], rows["level_loop"]))
    D.dawn_graph_release(ctx, h)
    return res


GRID_MEDIUM = dict(medium_edges=16384, medium_groups=32, blocks_per_cu=0)


def grid_bench(D, ctx, k_src=16):
    """The damaged 2048^2 grid (about 120 levels) under each level-loop
    driver, and the no-shortcut grid (thousands of levels) under two; driver
    3 also with medium push levels run on a few workgroups per launch."""
    import torch
    import graphgen as gg
    res = {}
    for name, drivers, ks in (("grid2048", (1, 2, 3, 4, "3m"), k_src), ("grid2048ns", (1, 3, "3m"), 1)):
        g, src = gg.load_config(name)
        h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        entry = {}
        for drv in drivers:
            kw = dict(driver=3 if drv == "3m" else drv, graph_levels=32, blocks_per_cu=1,
                      medium_edges=0)
            if drv == "3m":
                kw.update(GRID_MEDIUM)
            D.dawn_set_params(ctx, h, **kw)
            D.dawn_sssp(ctx, h, int(src[0]), out=out)
            t0 = time.perf_counter()
            se, lv = 0, []
            for s in src[:ks]:
                _, st = D.dawn_sssp(ctx, h, int(s), out=out)
                se += st["source_edges"]
                lv.append(st["levels"])
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            entry["driver3_medium" if drv == "3m" else f"driver{drv}"] = {
                "ms_per_source": round(t / ks * 1e3, 3), "gteps": round(se / t / 1e9, 3),
                "us_per_level": round(t / sum(lv) * 1e6, 2), "levels": lv}
        res[name] = entry
        D.dawn_graph_release(ctx, h)
    return res


def serve_run(D, ctx, graphs, queries, arrivals=None, window=48, host_out=False, keep_rows=0,
              skip=0):
    """Submit `queries` [(graph index, sources)], at `arrivals` (seconds from
    start; None = keep `window` queries in flight), and collect latencies
    (submit -> done) of every query after the first `skip`.  host_out: rows
    go to host arrays.  keep_rows: the first rows of each query are kept
    (host copies) for a parity check.  Returns (seconds, latencies ms, source
    edges, sources, graph index per latency, kept rows)."""
    import torch
    t0 = time.perf_counter()
    inflight = {}
    lat, gis, se, ks, kept = [], [], 0, 0, []
    i = 0
    t_first = None
    while i < len(queries) or inflight:
        now = time.perf_counter() - t0
        while i < len(queries) and (
                (arrivals is None and len(inflight) < window) or
                (arrivals is not None and arrivals[i] <= now)):
            gi, srcs = queries[i]
            h, g, esum = graphs[gi]
            if host_out:
                out = np.empty((srcs.size, g.n), np.int32)
            else:
                out = torch.empty((srcs.size, g.n), dtype=torch.int32, device="cuda")
            t = D.dawn_serve_submit(ctx, h, srcs, out)
            inflight[t] = (out, int(esum[srcs].sum()), srcs.size, gi, i)
            i += 1
        progressed = False
        for t in list(inflight):
            st, q = D.dawn_serve_poll(ctx, t)
            if st == D.DAWN_OK:
                out, e, k, gi, qi = inflight.pop(t)
                if qi >= skip:
                    if t_first is None:
                        t_first = q["submit_ns"]
                    lat.append((q["done_ns"] - q["submit_ns"]) / 1e6)
                    gis.append(gi)
                    se += e
                    ks += k
                if keep_rows:
                    # a device-side copy: no host wait inside the timed loop
                    r = out[:keep_rows]
                    kept.append((qi, r.copy() if host_out else r.clone()))
                progressed = True
        if not progressed:
            time.sleep(0.0002)
    dt = time.perf_counter() - t0
    kept = [(qi, r if isinstance(r, np.ndarray) else r.cpu().numpy()) for qi, r in kept]
    # the served rows were torch allocations: hand their cached blocks back so
    # that the library's own allocations (host-output staging) find the memory
    torch.cuda.empty_cache()
    return dt, np.array(lat), se, ks, np.array(gis), kept


def _per_graph(names, lat, gis):
    return {name: {"queries": int((gis == i).sum()),
                   "p50_ms": round(float(np.percentile(lat[gis == i], 50)), 3),
                   "p99_ms": round(float(np.percentile(lat[gis == i], 99)), 3)}
            for i, name in enumerate(names) if (gis == i).any()}


def serving_bench(D, ctx, nq=2000, skip=100, seed=105, keep=2, nq_host=300):
    """Three resident graphs, queries of 1..1024 sources (log-uniform) on a
    uniformly chosen graph, sources from its largest WCC: first saturated (a
    window of queries in flight) to find the capacity, then Poisson arrivals
    at 0.5 and 0.9 of that query rate; then the same with host-destination
    rows (saturated, then 0.5 of that mode's own rate).
    Each run submits `nq` queries and discards the first `skip` as warm-up
    (the host-destination run: the first `nq_host` of them, discarding a
    tenth; its rows, ~0.6 GB per query on the 2^20-node graphs, cross PCIe
    into fresh host pages).
    The first `keep` rows of every query of the saturated run are returned
    for the oracle check."""
    import graphgen as gg
    graphs = []
    names = ("rmat16", "rmat20", "grid1024")
    for name in names:
        g, _ = gg.load_config(name)
        h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
        graphs.append((h, g, component_edge_sums(g)))
    rng = np.random.default_rng(seed)
    queries = []
    for _ in range(nq):
        gi = int(rng.integers(0, 3))
        k = int(np.floor(np.exp(rng.uniform(0, np.log(1025)))))
        k = max(1, min(k, 1024))
        pool = graphs[gi][1].meta["wcc_nodes"]
        queries.append((gi, rng.choice(pool, size=k, replace=False).astype(np.int32)))
    serve_run(D, ctx, graphs, queries[:20])
    dt, lat, se, ks, gis, kept = serve_run(D, ctx, graphs, queries, skip=skip, keep_rows=keep)
    cap_qps = len(queries) / dt
    _log(f"[bench]   saturated: {len(queries)} queries in {dt:.1f} s")
    res = {"graphs": list(names), "queries": nq, "warmup_discarded": skip,
           "mean_k": round(float(np.mean([q[1].size for q in queries])), 1),
           "saturated": {"qps": round(cap_qps, 1), "sources_per_s": round(ks / dt, 1),
                         "gteps": round(se / dt / 1e9, 2),
                         "p50_ms": round(float(np.percentile(lat, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat, 99)), 3),
                         "per_graph": _per_graph(names, lat, gis)}}
    _log("[bench]   saturated, host output")
    dt, lat, se, ks, gis, _ = serve_run(D, ctx, graphs, queries[:nq_host], skip=nq_host // 20,
                                        host_out=True)
    cap_host = nq_host / dt
    res["saturated_host_output"] = {"queries": nq_host, "qps": round(cap_host, 1),
                                    "gteps": round(se / dt / 1e9, 2),
                                    "p50_ms": round(float(np.percentile(lat, 50)), 3),
                                    "p99_ms": round(float(np.percentile(lat, 99)), 3),
                                    "per_graph": _per_graph(names, lat, gis)}
    for label, frac, host in (("load_0.5", 0.5, False), ("load_0.9", 0.9, False),
                              ("load_0.5_host_output", 0.5, True)):
        lam = frac * (cap_host if host else cap_qps)
        nrun = nq_host if host else nq
        arr = np.cumsum(rng.exponential(1.0 / lam, size=nrun))
        dt, lat, se, ks, gis, _ = serve_run(D, ctx, graphs, queries[:nrun], arrivals=arr,
                                            skip=nrun // 20 if host else skip, host_out=host)
        _log(f"[bench]   {label}: {nrun} queries in {dt:.1f} s")
        res[label] = {"queries": nrun, "offered_qps": round(lam, 1),
                      "gteps": round(se / dt / 1e9, 2),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "per_graph": _per_graph(names, lat, gis)}
    used, budget = D.dawn_memory(ctx)
    res["hbm_used_gb"] = round(used / 1e9, 2)
    for h, _, _ in graphs:
        D.dawn_graph_release(ctx, h)
    check = [(graphs[queries[qi][0]][1], queries[qi][1][:keep], rows) for qi, rows in kept]
    return res, check


def served_parity(check):
    """The kept served rows against the oracle's rows for their sources."""
    import oracle
    bad, rows = 0, 0
    by_graph = {}
    for g, srcs, got in check:
        by_graph.setdefault(id(g), (g, [], []))
        by_graph[id(g)][1].append(srcs)
        by_graph[id(g)][2].append(got)
    for g, srcs, got in by_graph.values():
        s = np.concatenate(srcs)
        want = oracle.mssp(g, s, threads=host_cores())
        have = np.concatenate(got)
        bad += int((have != want).any(axis=1).sum())
        rows += int(s.size)
    return {"rows_checked": rows, "rows_differing": bad, "bit_exact": bad == 0}


def cpu_baseline(g, src):
    """The CPU oracle on the host cores: one thread, then one source per thread."""
    import oracle
    import graphgen as gg
    t0 = time.perf_counter()
    ref = oracle.mssp(g, src, threads=1)
    tc = time.perf_counter() - t0
    se = gg.reach_edges_from_dist(g, ref)
    cores = host_cores()
    t0 = time.perf_counter()
    oracle.mssp(g, src, threads=cores)
    tm = time.perf_counter() - t0
    base = {"value": round(se / tc / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"rmat20, the {src.size} timed sources, FIFO-queue BFS one source at a "
                      f"time, {tc:.1f} s",
            "cpu_model": cpu_model(), "host_cores": cores}
    par = {"value": round(se / tm / 1e9, 4), "unit": "GTEPS", "cores": cores, "kind": "oracle",
           "sample": f"same sources, one source per thread, {tm:.1f} s"}
    return base, par, ref


def host_dawn_bench(g, src, threads=(1, 2, 4, 8, 16), per=16):
    """The host CPU DAWN (SOVM on CPU threads) on R-MAT 20: one source at a
    time with N threads sharing each level, and the thread efficiency of the
    paper's scalability section, eta_N = T_1 / (T_N x N); then 64 sources
    spread one per thread."""
    from paper_2208_04514_amd import dawn_host as H
    hg = H.HostGraph(g.row_ptr, g.col)
    cores = host_cores()
    res, t1 = {}, None
    row = np.empty(g.n, np.int32)
    for nt in threads:
        if nt > cores:
            continue
        H.dawn_host_sssp(hg, int(src[0]), nt, out=row)
        t0 = time.perf_counter()
        se = 0
        for s in src[:per]:
            _, st = H.dawn_host_sssp(hg, int(s), nt, out=row)
            se += st["source_edges"]
        t = (time.perf_counter() - t0) / per
        t1 = t if nt == 1 else t1
        res[str(nt)] = {"ms_per_source": round(t * 1e3, 2), "gteps": round(se / per / t / 1e9, 4),
                        "efficiency": round(t1 / (t * nt), 4) if t1 else None}
    nt = min(16, cores)
    t0 = time.perf_counter()
    _, st = H.dawn_host_mssp(hg, src, nt)
    t = time.perf_counter() - t0
    hg.close()
    return {"workload": f"rmat20, {per} sources per thread count (one at a time); "
                        f"{src.size} sources one per thread", "per_source": res,
            "sources_parallel": {"threads": nt, "ms": round(t * 1e3, 1),
                                 "gteps": round(st["source_edges"] / t / 1e9, 4)},
            "host_cores": cores, "cpu_model": cpu_model()}


def roofline_only(D, ctx, params_json):
    """The level-kernel measurement alone (for profiling), then a 1 GiB device
    copy whose counters calibrate FETCH_SIZE and WRITE_SIZE."""
    import torch
    import graphgen as gg
    g, src = gg.load_config("rmat20")
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    out = torch.empty((src.size, g.n), dtype=torch.int32, device="cuda")
    if params_json:
        p = json.loads(params_json)
        D.dawn_set_params(ctx, h, **p)
    else:
        p, _, _ = cached_knobs(D, ctx, h, g, 1, PLAIN_KNOB_NAMES, 1, 9001, 32, False, None)
    lk_ms, lk_launches, levels, lk_clk = level_kernel_timing(D, ctx, h, src, out)
    torch.cuda.synchronize()
    roof = roofline_entry(g, out.cpu().numpy(), lk_ms, lk_launches, levels, p, lk_clk)
    # counter calibration: 1 GiB written, then copied (read 1 GiB, write 1 GiB);
    # the source is 4x the 256 MiB memory-side cache, so the copy reads HBM
    a = torch.empty(256 << 20, dtype=torch.int32, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"roofline": roof, "digest": kernel_digest(), "params": p,
                      "calibration_copy_read_bytes": a.numel() * 4,
                      "calibration_copy_write_bytes": b.numel() * 4}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the APSP and grid sections")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="search the knobs live (and record them) instead of loading the cache")
    ap.add_argument("--tune-file", default=None,
                    help="tuning cache to read and write (default: the package's tuned_params.json)")
    ap.add_argument("--tune-only", action="store_true",
                    help="search the knobs of the R-MAT 20 and R-MAT 18 workloads, record them in "
                         "the tuning cache, and stop")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the level-kernel timing pass (for rocprofv3)")
    ap.add_argument("--params", default="", help="JSON knobs for --roofline-only")
    ap.add_argument("--digest", action="store_true", help="print the level kernel's source digest")
    ap.add_argument("--batched-only", action="store_true",
                    help="only R-MAT 18 x 4096 sources through dawn_mssp, 3 calls (for profiling)")
    ap.add_argument("--grid-only", action="store_true",
                    help="only the grid2048 section (four sources per driver), for profilers")
    args = ap.parse_args()
    if args.digest:
        print(kernel_digest())
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the method shards over sources (no collectives), "
              "and this build runs and reports the single-GPU path only; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as gg
    from paper_2208_04514_amd import dawn as D

    if args.tune_only:
        ctx = D.dawn_create(0, 0)
        for name, width, names, what, seed, k in (
                ("rmat20", 1, PLAIN_KNOB_NAMES, 1, 9001, 32),
                ("rmat18", 4096, PLAIN_KNOB_NAMES + BATCH_KNOB_NAMES, 3, 9002, 4096)):
            g, _ = gg.load_config(name)
            h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
            knobs, _, s = cached_knobs(D, ctx, h, g, width, names, what, seed, k, True,
                                       args.tune_file)
            D.dawn_graph_release(ctx, h)
            _log(f"[tune] {name} width {width}: {json.dumps(knobs)} ({s:.1f} s)")
        return
    if args.roofline_only:
        ctx = D.dawn_create(0, 0)
        roofline_only(D, ctx, args.params)
        return
    if args.batched_only:
        ctx = D.dawn_create(0, 0)
        batched_only(D, ctx)
        return
    if args.grid_only:
        # the grid section alone (four grid2048 sources per driver), for a profiler
        ctx = D.dawn_create(0, 0)
        print(json.dumps({"grid_only": grid_bench(D, ctx, k_src=4)}), flush=True)
        return

    _log("[bench] R-MAT 20")
    g, src = gg.load_config("rmat20")
    ctx = D.dawn_create(0, 0)
    h = D.dawn_graph_upload(ctx, g.row_ptr, g.col)
    out = torch.empty((src.size, g.n), dtype=torch.int32, device="cuda")

    knobs, knobs_from, tune_s = cached_knobs(D, ctx, h, g, 1, PLAIN_KNOB_NAMES, 1, 9001, 32,
                                             args.autotune, args.tune_file)

    _log("[bench] plain SSSP timed region")
    se, dt, ks, levels, calls = run_plain(D, ctx, h, src, out, args.steps, args.warmup)
    value = se / dt / 1e9
    ms_per_step = dt / args.steps * 1e3
    timed_rows = out.cpu().numpy()          # the rows of the last timed pass

    _log("[bench] plain SSSP, host-destination rows (end to end, with the copy)")
    host_rows = np.empty((src.size, g.n), np.int32)
    t0 = time.perf_counter()
    se_h = 0
    for i, s in enumerate(src):
        _, st = D.dawn_sssp(ctx, h, int(s), out=host_rows[i])
        se_h += st["source_edges"]
    gteps_host = se_h / (time.perf_counter() - t0) / 1e9

    _log("[bench] level kernel per-launch timing")
    lk_ms, lk_launches, lk_levels, lk_clk = level_kernel_timing(D, ctx, h, src, out)
    torch.cuda.synchronize()
    dist_rows = out.cpu().numpy()           # the rows of the per-launch timing pass
    roofline = roofline_entry(g, dist_rows, lk_ms, lk_launches, lk_levels, knobs, lk_clk)
    bytes_full = D.dawn_graph_get_info(ctx, h)["device_bytes"]
    D.dawn_graph_release(ctx, h)

    extra = {}
    if not args.no_extra:
        _log("[bench] memory-frugal resident form (CSR shared as CSC)")
        hs = D.dawn_graph_upload(ctx, g.row_ptr, g.col, flags=D.DAWN_SHARED_CSC)
        D.dawn_set_params(ctx, hs, **knobs)
        se_s, dt_s, _, _, _ = run_plain(D, ctx, hs, src, out, 1, 1)
        extra["frugal"] = {"device_bytes": bytes_full,
                           "device_bytes_shared_csc": D.dawn_graph_get_info(ctx, hs)["device_bytes"],
                           "plain_gteps_shared_csc": round(se_s / dt_s / 1e9, 3),
                           "bit_exact_vs_full": bool(np.array_equal(out.cpu().numpy(), dist_rows))}
        D.dawn_graph_release(ctx, hs)

    if not args.no_batched:
        _log("[bench] batched R-MAT 18, 4096 sources")
        extra["batched"] = batched_bench(D, ctx, args.autotune, args.tune_file)
    if not args.no_extra:
        _log("[bench] uniform n = 4096, 8 sources")
        uniform_rows, extra["uniform4096"] = uniform_bench(D, ctx)
        _log("[bench] APSP over the largest WCC of R-MAT 14")
        extra["apsp"] = apsp_bench(D, ctx)
        _log("[bench] grid 2048^2 level-loop drivers")
        extra["grid"] = grid_bench(D, ctx)
        _log("[bench] weighted graphs ((min, +) level loop)")
        extra["weighted"] = weighted_bench(D, ctx)
        _log("[bench] small components")
        extra["small_components"] = small_component_bench(D, ctx)
    if not args.no_serve:
        _log("[bench] serving: R-MAT 16, R-MAT 20, grid 1024^2")
        extra["served"], served_check = serving_bench(D, ctx)

    cpu = None
    if not args.no_cpu:
        _log(f"[bench] CPU oracle on {src.size} sources")
        cpu, cpu_par, ref = cpu_baseline(g, src)
        extra["cpu_parallel"] = cpu_par
        # the oracle's rows against the rows of the timed pass itself, the
        # per-launch timing pass and the host-destination pass
        if not args.no_extra:
            import oracle
            gu, su = gg.load_config("uniform4096")
            extra["uniform4096"]["bit_exact"] = bool(np.array_equal(uniform_rows,
                                                                    oracle.mssp(gu, su)))
        if not args.no_serve:
            _log("[bench] oracle on the kept served rows")
            extra["served"]["parity"] = served_parity(served_check)
        if "batched" in extra:
            # the oracle on 256 of the batch's sources, one per host thread, and
            # those rows of the timed batched call against it
            gb, sb, kept = extra["batched"].pop("_kept")
            import oracle
            cores = host_cores()
            t0 = time.perf_counter()
            want = oracle.mssp(gb, sb, threads=cores)
            tb_cpu = time.perf_counter() - t0
            seb = gg.reach_edges_from_dist(gb, want)
            extra["batched"]["cpu_parallel_sample"] = {
                "value": round(seb / tb_cpu / 1e9, 4), "unit": "GTEPS", "cores": cores,
                "kind": "oracle", "sample": f"rmat18, 256 of the 4096 batch sources, one per "
                                            f"thread, {tb_cpu:.1f} s"}
            extra["batched"]["sample_rows_bit_exact"] = bool(np.array_equal(want, kept))
        extra["parity"] = {"timed_pass_bit_exact": bool(np.array_equal(ref, timed_rows)),
                           "timing_pass_bit_exact": bool(np.array_equal(ref, dist_rows)),
                           "host_output_bit_exact": bool(np.array_equal(ref, host_rows)),
                           "rows": int(src.size)}
        _log("[bench] host CPU DAWN (SOVM on CPU threads)")
        extra["host_dawn"] = host_dawn_bench(g, src)

    line = {
        "metric": "GTEPS (source-edge traversals/s), plain per-source SSSP",
        "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "rmat20_ef16_sym_64src_plain_sssp", "n": g.n, "m": g.m,
                   "sources": int(src.size), "source_edges_per_step": int(se // args.steps),
                   "gteps_device": round(se / ks / 1e6, 3),
                   "gteps_host_output": round(gteps_host, 3),
                   "gteps_graph500_halved": round(value / 2, 3),
                   "ms_per_source_p50": round(float(np.percentile(calls, 50)), 4),
                   "ms_per_source_p99": round(float(np.percentile(calls, 99)), 4),
                   "levels": int(np.max(levels)), "knobs": knobs,
                   "knobs_from": knobs_from,
                   "autotune_s": round(tune_s, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "batched" in extra:
        extra["batched"].pop("_kept", None)
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
