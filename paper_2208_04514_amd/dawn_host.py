"""Thin ctypes binding of ``libdawn_host.so`` (the C ABI in ``include/dawn_host.h``):
DAWN's SOVM level loop on the host's CPU cores.  Same function names; argument
marshalling only.  Separate from the GPU library."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdawn_host.so")


class HostStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("source_edges", ctypes.c_int64),
                ("reached", ctypes.c_int64), ("ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class DawnHostError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


_LIB = None


def load(path: str | None = None):
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"libdawn_host.so not built at {path}: run python -m paper_2208_04514_amd.host.build")
    L = ctypes.CDLL(path)
    V, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.dawn_host_graph_create.argtypes = [I32, I64, V, V, ctypes.POINTER(V)]
    L.dawn_host_graph_destroy.argtypes = [V]
    L.dawn_host_sssp.argtypes = [V, I32, I32, V, ctypes.POINTER(HostStats)]
    L.dawn_host_mssp.argtypes = [V, V, I32, I32, V, ctypes.POINTER(HostStats)]
    for f in ("dawn_host_graph_create", "dawn_host_graph_destroy", "dawn_host_sssp", "dawn_host_mssp"):
        getattr(L, f).restype = I32
    L.dawn_host_last_error.restype = ctypes.c_char_p
    _LIB = L
    return L


def _check(st: int):
    if st != 0:
        raise DawnHostError(st, load().dawn_host_last_error().decode())
    return st


class HostGraph:
    """A CSR graph wrapped for the host library (keeps the arrays alive)."""

    def __init__(self, row_ptr, col):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.n = self.row_ptr.size - 1
        h = ctypes.c_void_p()
        _check(load().dawn_host_graph_create(self.n, self.col.size, self.row_ptr.ctypes.data,
                                             self.col.ctypes.data if self.col.size else None,
                                             ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            load().dawn_host_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dawn_host_sssp(g: HostGraph, source: int, threads: int = 1, out=None):
    """(dist int32[n], stats dict)."""
    dist = np.empty(g.n, np.int32) if out is None else out
    st = HostStats()
    _check(load().dawn_host_sssp(g.handle, int(source), int(threads), dist.ctypes.data, ctypes.byref(st)))
    return dist, st.as_dict()


def dawn_host_mssp(g: HostGraph, sources, threads: int = 1, out=None):
    """(dist int32[k, n], stats dict); row r is sources[r]."""
    src = np.ascontiguousarray(sources, dtype=np.int32)
    dist = np.empty((src.size, g.n), np.int32) if out is None else out
    st = HostStats()
    _check(load().dawn_host_mssp(g.handle, src.ctypes.data if src.size else None, src.size, int(threads),
                                 dist.ctypes.data if src.size else None, ctypes.byref(st)))
    return dist, st.as_dict()
