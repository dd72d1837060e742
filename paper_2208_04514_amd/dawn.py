"""Thin ctypes binding of ``libdawn.so`` (the C ABI in ``include/dawn.h``).

Functions carry the C entry points' names and only marshal arguments: every
step of the traversal runs in the library's HIP kernels.  Host outputs are
numpy arrays; device outputs are torch CUDA tensors (their ``data_ptr()`` is
passed with ``DAWN_DEVICE_OUT``).  There is no fallback: if the library is not
built, :func:`load` raises.
"""
from __future__ import annotations

import ctypes
import os
import struct

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdawn.so")

DAWN_OK = 0
DAWN_PENDING = 1
DAWN_E_INVALID_ARG = -1
DAWN_E_BAD_GRAPH = -2
DAWN_E_NO_MEMORY = -3
DAWN_E_DEVICE = -4
DAWN_E_NOT_FOUND = -5
DAWN_E_BUSY = -6
DAWN_DEVICE_OUT = 0x1
DAWN_SHARED_CSC = 0x2

STATUS_NAMES = {
    0: "DAWN_OK", 1: "DAWN_PENDING", -1: "DAWN_E_INVALID_ARG", -2: "DAWN_E_BAD_GRAPH",
    -3: "DAWN_E_NO_MEMORY", -4: "DAWN_E_DEVICE", -5: "DAWN_E_NOT_FOUND", -6: "DAWN_E_BUSY",
}

EXPORTED = (
    "dawn_create", "dawn_destroy", "dawn_last_error", "dawn_memory", "dawn_graph_upload",
    "dawn_graph_release", "dawn_graph_get_info", "dawn_get_params", "dawn_set_params",
    "dawn_sssp", "dawn_mssp", "dawn_apsp_wcc", "dawn_autotune", "dawn_serve_submit",
    "dawn_serve_poll", "dawn_serve_wait", "dawn_mssp_device", "dawn_sssp_noalloc",
    "dawn_graph_set_weights", "dawn_sssp_weighted",
)


class DawnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class RunStats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("push_levels", ctypes.c_int32),
        ("pull_levels", ctypes.c_int32), ("launches", ctypes.c_int32),
        ("edges_examined", ctypes.c_int64), ("source_edges", ctypes.c_int64),
        ("reached", ctypes.c_int64), ("kernel_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double), ("frontier_sizes", _i32p),
        ("directions", _u8p), ("frontier_cap", ctypes.c_int32),
        ("kernel_clock_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        # the first nine fields in one unpack of the structure's bytes (a
        # getattr per field costs about a microsecond per call in all)
        d = dict(zip(_RUN_STATS_HEAD, _RUN_STATS_UNPACK.unpack_from(self)))
        d["kernel_clock_ms"] = self.kernel_clock_ms
        return d


_RUN_STATS_HEAD = tuple(f for f, _ in RunStats._fields_[:9])
_RUN_STATS_UNPACK = struct.Struct("=4i3q2d")   # levels .. total_ms, no padding between them
assert _RUN_STATS_UNPACK.size == RunStats.total_ms.offset + 8


class Params(ctypes.Structure):
    _fields_ = [
        ("driver", ctypes.c_int32), ("direction", ctypes.c_int32), ("block", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32), ("big_degree", ctypes.c_int32),
        ("pull_lane_edges", ctypes.c_int32), ("alpha", ctypes.c_float),
        ("beta", ctypes.c_float), ("graph_levels", ctypes.c_int32),
        ("small_n", ctypes.c_int32), ("batch_alpha", ctypes.c_float),
        ("batch_lanes", ctypes.c_int32), ("timing", ctypes.c_int32),
        ("batch_big_degree", ctypes.c_int32), ("batch_wide_scan", ctypes.c_int32),
        ("batch_sparse_words", ctypes.c_int32), ("small_frontier_edges", ctypes.c_int32),
        ("medium_edges", ctypes.c_int32), ("medium_groups", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class GraphInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("max_out_degree", ctypes.c_int32), ("m", ctypes.c_int64),
        ("zero_out_degree", ctypes.c_int32), ("s_wcc", ctypes.c_int32),
        ("device_bytes", ctypes.c_int64),
    ]


class QueryStats(ctypes.Structure):
    _fields_ = [
        ("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64),
        ("done_ns", ctypes.c_uint64), ("levels", ctypes.c_int32), ("status", ctypes.c_int32),
        ("k", ctypes.c_int32), ("batch_peak", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_LIB = None


def load(path: str | None = None):
    """Load the built library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or LIB_PATH
    # torch bundles its own HIP runtime under the same SONAME; importing torch
    # first makes libdawn bind to that copy, so a process never holds two HIP
    # runtimes (the second one could not open the GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(f"libdawn.so not built at {path}: run python -m paper_2208_04514_amd.build")
    L = ctypes.CDLL(path)
    V, I32, I64, U32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "dawn_create": [I32, U64, ctypes.POINTER(V)],
        "dawn_destroy": [V],
        "dawn_memory": [V, ctypes.POINTER(U64), ctypes.POINTER(U64)],
        "dawn_graph_upload": [V, I32, I64, V, V, U32, _i32p],
        "dawn_graph_release": [V, I32],
        "dawn_graph_get_info": [V, I32, ctypes.POINTER(GraphInfo)],
        "dawn_get_params": [V, I32, ctypes.POINTER(Params)],
        "dawn_set_params": [V, I32, ctypes.POINTER(Params)],
        "dawn_sssp": [V, I32, I32, V, U32, ctypes.POINTER(RunStats)],
        "dawn_mssp": [V, I32, V, I32, V, U32, ctypes.POINTER(RunStats)],
        "dawn_apsp_wcc": [V, I32, V, _i32p, V, U32, ctypes.POINTER(RunStats)],
        "dawn_autotune": [V, I32, V, I32, U32, ctypes.POINTER(Params)],
        "dawn_serve_submit": [V, I32, V, I32, V, U32, ctypes.POINTER(U64)],
        "dawn_serve_poll": [V, U64, ctypes.POINTER(QueryStats)],
        "dawn_serve_wait": [V, U64, I32, ctypes.POINTER(QueryStats)],
        "dawn_mssp_device": [V, I32, V, I32, V, V, V],
        "dawn_sssp_noalloc": [V, I32, I32, V, V, ctypes.POINTER(RunStats)],
        "dawn_graph_set_weights": [V, I32, V],
        "dawn_sssp_weighted": [V, I32, I32, V, U32, ctypes.POINTER(RunStats)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I32
    L.dawn_last_error.argtypes = []
    L.dawn_last_error.restype = ctypes.c_char_p
    _LIB = L
    return L


def _check(st: int, allow=(DAWN_OK,)) -> int:
    if st not in allow:
        msg = load().dawn_last_error().decode(errors="replace")
        raise DawnError(st, msg)
    return st


def dawn_last_error() -> str:
    return load().dawn_last_error().decode(errors="replace")


# ------------------------------------------------------------------ helpers --

def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


def _is_torch_cuda(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


# Facts the binding keeps per context and graph, so that an output buffer can
# be checked against what the library will write before the call is made:
# the device of each context, and n of each resident graph (ids are never
# reused within a context).
_CTX_DEVICE: dict[int, int] = {}
_GRAPH_N: dict[tuple[int, int], int] = {}


def _ctx_key(ctx) -> int:
    return int(ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx or 0)


def _graph_n(ctx, graph: int) -> int:
    key = (_ctx_key(ctx), int(graph))
    n = _GRAPH_N.get(key)
    if n is None:
        n = dawn_graph_get_info(ctx, graph)["n"]
        _GRAPH_N[key] = n
    return n


def check_out(out, shape: tuple, device: int | None = None):
    """Validate an output buffer for a call that writes ``prod(shape)`` int32.

    ``out`` must hold exactly that many elements (its shape may be flat or
    ``shape``): a host ``numpy`` int32 C-contiguous array, or a contiguous
    int32 torch CUDA tensor on ``device`` (the context's GPU).  Returns
    ``(pointer, flags, keepalive)``; raises ``ValueError`` before any library
    call when the buffer does not match.
    """
    count = 1
    for d in shape:
        count *= int(d)
    if _is_torch_cuda(out):
        import torch
        if out.dtype != torch.int32 or not out.is_contiguous():
            raise ValueError("device output must be a contiguous int32 CUDA tensor")
        if out.numel() != count or (out.dim() > 1 and tuple(out.shape) != tuple(shape)):
            raise ValueError(f"device output has shape {tuple(out.shape)}, the call writes {tuple(shape)}")
        if device is not None and out.device.index != device:
            raise ValueError(f"device output is on cuda:{out.device.index}, the context on cuda:{device}")
        return ctypes.c_void_p(out.data_ptr()), DAWN_DEVICE_OUT, out
    if not (isinstance(out, np.ndarray) and out.dtype == np.int32 and out.flags.c_contiguous
            and out.flags.writeable):
        raise ValueError("host output must be a writeable C-contiguous int32 numpy array")
    if out.size != count or (out.ndim > 1 and out.shape != tuple(shape)):
        raise ValueError(f"host output has shape {out.shape}, the call writes {tuple(shape)}")
    return out.ctypes.data_as(ctypes.c_void_p), 0, out


def _out_ptr(ctx, out, shape: tuple):
    """check_out against the context's device; a synchronous call with device
    output first lets pending torch work on the caller's stream finish (the
    library writes on its own streams)."""
    ptr, flags, keep = check_out(out, shape, _CTX_DEVICE.get(_ctx_key(ctx)))
    if flags & DAWN_DEVICE_OUT:
        import torch
        torch.cuda.current_stream(out.device).synchronize()
    return ptr, flags, keep


# -------------------------------------------------------------- entry points --

def dawn_create(device: int = 0, hbm_budget_bytes: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().dawn_create(device, hbm_budget_bytes, ctypes.byref(h)))
    _CTX_DEVICE[_ctx_key(h)] = int(device)
    return h


def dawn_destroy(ctx) -> None:
    key = _ctx_key(ctx)
    _check(load().dawn_destroy(ctx))
    _CTX_DEVICE.pop(key, None)
    for gk in [gk for gk in _GRAPH_N if gk[0] == key]:
        del _GRAPH_N[gk]


def dawn_memory(ctx) -> tuple[int, int]:
    u, b = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().dawn_memory(ctx, ctypes.byref(u), ctypes.byref(b)))
    return u.value, b.value


def dawn_graph_upload(ctx, row_ptr, col, flags: int = 0) -> int:
    rp = _host_i32(row_ptr)
    c = _host_i32(col)
    n = rp.size - 1
    g = ctypes.c_int32(-1)
    _check(load().dawn_graph_upload(ctx, n, int(c.size), rp.ctypes.data_as(ctypes.c_void_p),
                                    c.ctypes.data_as(ctypes.c_void_p) if c.size else None,
                                    flags, ctypes.byref(g)))
    _GRAPH_N[(_ctx_key(ctx), g.value)] = n
    return g.value


def dawn_graph_set_weights(ctx, graph: int, weights) -> None:
    """Attach int32 weights (one per CSR entry, >= 0) to a resident graph."""
    w = _host_i32(weights).ravel()
    m = dawn_graph_get_info(ctx, graph)["m"]
    if w.size != m:
        raise ValueError(f"{w.size} weights for a graph of {m} edges")
    _check(load().dawn_graph_set_weights(ctx, graph, w.ctypes.data_as(ctypes.c_void_p)
                                         if w.size else None))


def dawn_sssp_weighted(ctx, graph: int, source: int, out=None):
    """Weighted distances from `source` ((min, +) level loop).  `out`: numpy
    int32[n] or torch int32 CUDA tensor.  Returns ``(out, stats)``."""
    n = _graph_n(ctx, graph)
    if out is None:
        out = np.empty(n, dtype=np.int32)
    ptr, flags, _keep = _out_ptr(ctx, out, (n,))
    st = RunStats()
    _check(load().dawn_sssp_weighted(ctx, graph, int(source), ptr, flags, ctypes.byref(st)))
    return out, st.as_dict()


def dawn_graph_release(ctx, graph: int) -> None:
    _check(load().dawn_graph_release(ctx, graph))
    _GRAPH_N.pop((_ctx_key(ctx), int(graph)), None)


def dawn_graph_get_info(ctx, graph: int) -> dict:
    info = GraphInfo()
    _check(load().dawn_graph_get_info(ctx, graph, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in GraphInfo._fields_}


def dawn_get_params(ctx, graph: int) -> dict:
    p = Params()
    _check(load().dawn_get_params(ctx, graph, ctypes.byref(p)))
    return p.as_dict()


def dawn_set_params(ctx, graph: int, **kw) -> dict:
    """Set knobs by name; unnamed knobs keep their current value."""
    cur = dawn_get_params(ctx, graph)
    cur.update(kw)
    p = Params(**cur)
    _check(load().dawn_set_params(ctx, graph, ctypes.byref(p)))
    return dawn_get_params(ctx, graph)


def dawn_sssp(ctx, graph: int, source: int, out=None, frontier_cap: int = 0):
    """Distances from `source`.  `out`: numpy int32[n] or torch int32 CUDA tensor.

    Returns ``(out, stats)``; with ``frontier_cap`` > 0 the stats dict also has
    ``frontier_sizes`` and ``directions`` lists.
    """
    n = _graph_n(ctx, graph)
    if out is None:
        out = np.empty(n, dtype=np.int32)
    ptr, flags, _keep = _out_ptr(ctx, out, (n,))
    st = RunStats()
    if frontier_cap > 0:
        fs = np.zeros(frontier_cap, np.int32)
        dr = np.zeros(frontier_cap, np.uint8)
        st.frontier_sizes = fs.ctypes.data_as(_i32p)
        st.directions = dr.ctypes.data_as(_u8p)
        st.frontier_cap = frontier_cap
    _check(load().dawn_sssp(ctx, graph, int(source), ptr, flags, ctypes.byref(st)))
    d = st.as_dict()
    if frontier_cap > 0:
        L = min(st.levels, frontier_cap)
        d["frontier_sizes"] = fs[:L].tolist()
        d["directions"] = dr[:L].tolist()
    return out, d


def dawn_sssp_noalloc(ctx, graph: int, source: int, out, stream=None):
    """Distances from `source` into the int32 CUDA tensor `out` [n], with no
    device allocation by the library (its static scratch array); the work is
    queued on `stream` (default: torch's current stream) and finished on
    return.  Returns ``(out, stats)``."""
    import torch
    ptr, _flags, _keep = check_out(out, (_graph_n(ctx, graph),), _CTX_DEVICE.get(_ctx_key(ctx)))
    if not _is_torch_cuda(out):
        raise ValueError("dawn_sssp_noalloc writes device memory: pass an int32 CUDA tensor")
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    st = RunStats()
    _check(load().dawn_sssp_noalloc(ctx, graph, int(source), ptr,
                                    ctypes.c_void_p(stream.cuda_stream), ctypes.byref(st)))
    return out, st.as_dict()


def dawn_mssp(ctx, graph: int, sources, out=None):
    """Row r = distances from sources[r].  `out`: int32 [k, n] numpy or torch CUDA."""
    src = _host_i32(sources).ravel()
    k = src.size
    n = _graph_n(ctx, graph)
    if out is None:
        out = np.empty((k, n), dtype=np.int32)
    ptr, flags, _keep = _out_ptr(ctx, out, (k, n))
    st = RunStats()
    _check(load().dawn_mssp(ctx, graph, src.ctypes.data_as(ctypes.c_void_p), k, ptr, flags,
                            ctypes.byref(st)))
    return out, st.as_dict()


def dawn_mssp_device(ctx, graph: int, sources, out, status=None, stream=None):
    """Queue a multi-source run on a torch stream (default: the current one).

    ``sources``: int32 CUDA tensor of k node ids; ``out``: int32 CUDA tensor
    [k, n]; ``status`` (optional): int32 CUDA tensor of one element that
    receives the run's status on the stream.  Returns at once: later work on
    the stream sees the rows; nothing here waits for the device.
    """
    import torch
    dev = _CTX_DEVICE.get(_ctx_key(ctx))
    if not (_is_torch_cuda(sources) and sources.dtype == torch.int32 and sources.is_contiguous()
            and sources.dim() == 1):
        raise ValueError("sources must be a contiguous 1-D int32 CUDA tensor")
    if dev is not None and sources.device.index != dev:
        raise ValueError(f"sources are on cuda:{sources.device.index}, the context on cuda:{dev}")
    k = int(sources.numel())
    ptr, _flags, _keep = check_out(out, (k, _graph_n(ctx, graph)), dev)
    sp = None
    if status is not None:
        sp, _f, _k = check_out(status, (1,), dev)
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    _check(load().dawn_mssp_device(ctx, graph, ctypes.c_void_p(sources.data_ptr()), k, ptr, sp,
                                   ctypes.c_void_p(stream.cuda_stream)))
    return out


def dawn_apsp_wcc(ctx, graph: int, out=None, query_only: bool = False):
    """(wcc_nodes, dist [s_wcc, s_wcc] or None, stats)."""
    nodes = np.empty(_graph_n(ctx, graph), np.int32)
    s = ctypes.c_int32(0)
    st = RunStats()
    lib = load()
    if query_only:
        _check(lib.dawn_apsp_wcc(ctx, graph, nodes.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(s), None, 0, ctypes.byref(st)))
        return nodes[: s.value].copy(), None, st.as_dict()
    # the component's size first: the call writes s_wcc x s_wcc
    _check(lib.dawn_apsp_wcc(ctx, graph, nodes.ctypes.data_as(ctypes.c_void_p),
                             ctypes.byref(s), None, 0, None))
    if out is None:
        out = np.empty((s.value, s.value), np.int32)
    ptr, flags, _keep = _out_ptr(ctx, out, (s.value, s.value))
    _check(lib.dawn_apsp_wcc(ctx, graph, nodes.ctypes.data_as(ctypes.c_void_p), ctypes.byref(s),
                             ptr, flags, ctypes.byref(st)))
    return nodes[: s.value].copy(), out, st.as_dict()


def dawn_autotune(ctx, graph: int, sources, what: int = 3) -> dict:
    src = _host_i32(sources)
    p = Params()
    _check(load().dawn_autotune(ctx, graph, src.ctypes.data_as(ctypes.c_void_p), src.size, what,
                                ctypes.byref(p)))
    return p.as_dict()


def dawn_serve_submit(ctx, graph: int, sources, out) -> int:
    """Queue a query; `out` (int32 [k, n], numpy or torch CUDA) must stay alive until done.

    The server writes a device `out` on its own stream, later: pending work
    on the caller's torch stream (a fill of `out`, say) is finished first, so
    it cannot land on top of the rows."""
    src = _host_i32(sources).ravel()
    ptr, flags, _keep = _out_ptr(ctx, out, (src.size, _graph_n(ctx, graph)))
    t = ctypes.c_uint64(0)
    _check(load().dawn_serve_submit(ctx, graph, src.ctypes.data_as(ctypes.c_void_p), src.size,
                                    ptr, flags, ctypes.byref(t)))
    return t.value


def dawn_serve_poll(ctx, ticket: int):
    """(status, stats dict): status is DAWN_OK or DAWN_PENDING; errors raise."""
    q = QueryStats()
    st = _check(load().dawn_serve_poll(ctx, ticket, ctypes.byref(q)), (DAWN_OK, DAWN_PENDING))
    return st, q.as_dict()


def dawn_serve_wait(ctx, ticket: int, timeout_ms: int = -1):
    q = QueryStats()
    st = _check(load().dawn_serve_wait(ctx, ticket, timeout_ms, ctypes.byref(q)),
                (DAWN_OK, DAWN_PENDING))
    return st, q.as_dict()
