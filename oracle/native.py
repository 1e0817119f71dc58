"""ctypes access to the oracle's C part: Dijkstra on a raw edge list, and the
CSR invariant checker. Test infrastructure only (see ``oracle/__init__.py``)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, BAD_ARGS, NOMEM, OVERFLOW = 0, -1, -2, 1
INF = 0xFFFFFFFF


def use_build(path: str) -> None:
    """Load another build of the same source (say one tuned for this host)
    in place of the in-tree library, for every later call."""
    global _lib
    _lib = None
    _load(path)


def _load(path: str = None):
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = _LIB_PATH
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
    lib = ctypes.CDLL(path)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64 = ctypes.c_int64
    lib.oracle_adj_build.argtypes = [i64, i64, i32p, i32p, u32p]
    lib.oracle_adj_build.restype = ctypes.c_void_p
    lib.oracle_adj_free.argtypes = [ctypes.c_void_p]
    lib.oracle_adj_free.restype = None
    lib.oracle_adj_dijkstra.argtypes = [ctypes.c_void_p, ctypes.c_int32, u32p]
    lib.oracle_adj_dijkstra.restype = ctypes.c_int
    lib.oracle_adj_dijkstra_many.argtypes = [ctypes.c_void_p, ctypes.c_int32, i32p, u32p, ctypes.c_int32]
    lib.oracle_adj_dijkstra_many.restype = ctypes.c_int
    lib.oracle_dijkstra.argtypes = [i64, i64, i32p, i32p, u32p, ctypes.c_int32, u32p]
    lib.oracle_dijkstra.restype = ctypes.c_int
    lib.oracle_check_sssp.argtypes = [i64, i32p, i32p, u32p, ctypes.c_int32, u32p,
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_check_sssp.restype = ctypes.c_int64
    lib.oracle_adj_dijkstra_f32.argtypes = [ctypes.c_void_p, ctypes.c_int32, u32p]
    lib.oracle_adj_dijkstra_f32.restype = ctypes.c_int
    lib.oracle_adj_dijkstra_tree.argtypes = [ctypes.c_void_p, ctypes.c_int32, u32p, i32p]
    lib.oracle_adj_dijkstra_tree.restype = ctypes.c_int
    lib.oracle_check_tree.argtypes = [i64, i32p, i32p, u32p, ctypes.c_int32, u32p, i32p,
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_check_tree.restype = ctypes.c_int64
    _lib = lib
    return lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class Adjacency:
    """Undirected adjacency of a raw edge list, built once, solved many times."""

    def __init__(self, n, src, dst, w):
        lib = _load()
        self._src = np.ascontiguousarray(src, np.int32)
        self._dst = np.ascontiguousarray(dst, np.int32)
        self._w = np.ascontiguousarray(w, np.uint32)
        self.n = int(n)
        self._h = lib.oracle_adj_build(self.n, self._src.shape[0], _p(self._src, ctypes.c_int32),
                                       _p(self._dst, ctypes.c_int32), _p(self._w, ctypes.c_uint32))
        if not self._h:
            raise ValueError("oracle_adj_build: bad edge list")

    def dijkstra(self, s: int) -> np.ndarray:
        out = np.empty(self.n, np.uint32)
        rc = _load().oracle_adj_dijkstra(self._h, int(s), _p(out, ctypes.c_uint32))
        if rc == OVERFLOW:
            raise OverflowError("a shortest-path length does not fit below 2^32-1")
        if rc != OK:
            raise RuntimeError("oracle_adj_dijkstra failed: %d" % rc)
        return out

    def dijkstra_f32(self, s: int) -> np.ndarray:
        """Binary32 weights (bit patterns) and distances: uint32 bit patterns,
        0xFFFFFFFF where unreachable."""
        out = np.empty(self.n, np.uint32)
        rc = _load().oracle_adj_dijkstra_f32(self._h, int(s), _p(out, ctypes.c_uint32))
        if rc != OK:
            raise RuntimeError("oracle_adj_dijkstra_f32 failed: %d" % rc)
        return out

    def dijkstra_tree(self, s: int):
        """Distances and the predecessor array (parent[s] = s, -1 where unreachable)."""
        out = np.empty(self.n, np.uint32)
        par = np.empty(self.n, np.int32)
        rc = _load().oracle_adj_dijkstra_tree(self._h, int(s), _p(out, ctypes.c_uint32), _p(par, ctypes.c_int32))
        if rc == OVERFLOW:
            raise OverflowError("a shortest-path length does not fit below 2^32-1")
        if rc != OK:
            raise RuntimeError("oracle_adj_dijkstra_tree failed: %d" % rc)
        return out, par

    def dijkstra_many(self, sources, threads: int) -> np.ndarray:
        srcs = np.ascontiguousarray(sources, np.int32)
        out = np.empty((srcs.shape[0], self.n), np.uint32)
        rc = _load().oracle_adj_dijkstra_many(self._h, srcs.shape[0], _p(srcs, ctypes.c_int32),
                                              _p(out, ctypes.c_uint32), int(threads))
        if rc != OK:
            raise RuntimeError("oracle_adj_dijkstra_many failed: %d" % rc)
        return out

    def close(self):
        if self._h:
            _load().oracle_adj_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dijkstra(n, src, dst, w, s) -> np.ndarray:
    """Exact distances from s over the raw undirected edge list (u32, INF = 2^32-1)."""
    a = Adjacency(n, src, dst, w)
    try:
        return a.dijkstra(s)
    finally:
        a.close()


def check_sssp(n, rowptr, col, w, s, dist):
    """Invariant violation counts of a candidate distance vector on a CSR:
    [d(s)!=0, improvable edges, no tight in-edge, not tight-reachable, inf next to finite]."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    w = np.ascontiguousarray(w, np.uint32)
    dist = np.ascontiguousarray(dist, np.uint32)
    counts = (ctypes.c_int64 * 5)()
    tot = lib.oracle_check_sssp(int(n), _p(rowptr, ctypes.c_int32), _p(col, ctypes.c_int32),
                                _p(w, ctypes.c_uint32), int(s), _p(dist, ctypes.c_uint32), counts)
    if tot < 0:
        raise ValueError("oracle_check_sssp: bad arguments")
    return [int(c) for c in counts]


def check_tree(n, rowptr, col, w, s, dist, parent):
    """Violation counts of a candidate predecessor array against a distance vector on a
    CSR: [parent(s) != s, bad entry (unreachable with a parent, or not a vertex id),
    parent edge not tight, chain not ending at s]."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    w = np.ascontiguousarray(w, np.uint32)
    dist = np.ascontiguousarray(dist, np.uint32)
    parent = np.ascontiguousarray(parent, np.int32)
    counts = (ctypes.c_int64 * 4)()
    tot = lib.oracle_check_tree(int(n), _p(rowptr, ctypes.c_int32), _p(col, ctypes.c_int32),
                                _p(w, ctypes.c_uint32), int(s), _p(dist, ctypes.c_uint32),
                                _p(parent, ctypes.c_int32), counts)
    if tot == -1:
        raise ValueError("oracle_check_tree: bad arguments")
    if tot < 0:
        raise MemoryError("oracle_check_tree: out of memory")
    return [int(c) for c in counts]
