"""Seeded synthetic inputs for the SSSP engine and its oracle.

Inputs only: this package holds none of the shortest-path method's arithmetic.
It draws undirected edge lists (R-MAT, G(n, m), road-like grid), cleans them
into a symmetric CSR (self-loops dropped, parallel edges merged to their
minimum weight, rows sorted by column) and picks sources uniformly among
vertices of degree >= 1 (the paper's trial protocol, Section 4, draws 64 such
sources per graph).

The heavy lifting is in ``gen.cpp`` (``libgraphgen.so``), built by
``graphgen/build.py``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# Seeds: 20250619 + workload index, recorded in every result.
SEED_BASE = 20250619


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64 = ctypes.c_int64
    lib.gg_rmat.argtypes = [ctypes.c_int32, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, i32p, i32p, u32p]
    lib.gg_rmat.restype = ctypes.c_int
    lib.gg_gnm.argtypes = [i64, i64, ctypes.c_uint32, ctypes.c_uint64, i32p, i32p, u32p]
    lib.gg_gnm.restype = ctypes.c_int
    lib.gg_weights_power.argtypes = [i64, ctypes.c_uint64, ctypes.c_int32, u32p]
    lib.gg_weights_power.restype = ctypes.c_int
    lib.gg_weights_f32.argtypes = [i64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, u32p]
    lib.gg_weights_f32.restype = ctypes.c_int
    lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_uint32, ctypes.c_uint64, i32p, i32p, u32p]
    lib.gg_grid.restype = i64
    lib.gg_csr_build.argtypes = [i64, i64, i32p, i32p, u32p, ctypes.POINTER(i64)]
    lib.gg_csr_build.restype = ctypes.c_void_p
    lib.gg_csr_copy.argtypes = [ctypes.c_void_p, i32p, i32p, u32p]
    lib.gg_csr_copy.restype = None
    lib.gg_csr_free.argtypes = [ctypes.c_void_p]
    lib.gg_csr_free.restype = None
    lib.gg_pick_sources.argtypes = [i64, i32p, ctypes.c_int32, ctypes.c_uint64, i32p]
    lib.gg_pick_sources.restype = ctypes.c_int32
    lib.gg_rmat_degrees.argtypes = [ctypes.c_int32, i64, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_uint64, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int64)]
    lib.gg_rmat_degrees.restype = ctypes.c_int
    lib.gg_permutation.argtypes = [i64, ctypes.c_uint64, i32p]
    lib.gg_permutation.restype = None
    _lib = lib
    return lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclasses.dataclass
class EdgeList:
    """Raw undirected edge list: may hold self-loops and parallel edges."""
    n: int
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    w: np.ndarray    # uint32[m]

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


@dataclasses.dataclass
class CSR:
    """Symmetric CSR: rowptr int32[n+1], col int32[nnz], w uint32[nnz]."""
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    w: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         wmax: int = 255, seed: int = SEED_BASE, relabel: bool = True) -> EdgeList:
    lib = _load()
    n = 1 << scale
    m = edge_factor << scale
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    w = np.empty(m, np.uint32)
    rc = lib.gg_rmat(scale, edge_factor, a, b, c, wmax, seed, int(relabel),
                     _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32), _p(w, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("gg_rmat: bad arguments")
    return EdgeList(n, src, dst, w)


def weights_power(m: int, power: int, seed: int) -> np.ndarray:
    """The integer-power variant weights (Eq. 7) of m edges: the integer
    nearest to 1 + x (2^power - 2), x uniform on (0, 1], halves rounded up."""
    lib = _load()
    w = np.empty(m, np.uint32)
    if lib.gg_weights_power(m, seed, power, _p(w, ctypes.c_uint32)) != 0:
        raise ValueError("gg_weights_power: bad arguments")
    return w


def weights_f32(m: int, seed: int, pivot: Optional[float] = None) -> np.ndarray:
    """Real weights as binary32 bit patterns (uint32): x uniform on (0, 1] (the
    gr26 graphs), or with a pivot the float-pivot variant converge(x, pivot)
    of Eq. 8."""
    lib = _load()
    w = np.empty(m, np.uint32)
    mode, p = (0, 0.5) if pivot is None else (1, float(pivot))
    if lib.gg_weights_f32(m, seed, mode, p, _p(w, ctypes.c_uint32)) != 0:
        raise ValueError("gg_weights_f32: bad arguments")
    return w


def rmat_degrees(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
                 c: float = 0.19, seed: int = SEED_BASE, relabel: bool = True) -> np.ndarray:
    """Degrees of the R-MAT multigraph (parallel edges counted, self-loops
    dropped) without materialising the edge list."""
    lib = _load()
    deg = np.empty(1 << scale, np.int64)
    rc = lib.gg_rmat_degrees(scale, edge_factor, a, b, c, seed, int(relabel),
                             deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("gg_rmat_degrees: bad arguments")
    return deg


def gnm(n: int, m: int, wmax: int = 255, seed: int = SEED_BASE) -> EdgeList:
    lib = _load()
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    w = np.empty(m, np.uint32)
    rc = lib.gg_gnm(n, m, wmax, seed, _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32),
                    _p(w, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("gg_gnm: bad arguments")
    return EdgeList(n, src, dst, w)


def grid(rows: int, cols: int, p_keep: float = 0.95, p_diag: float = 0.01, wmax: int = 1000,
         seed: int = SEED_BASE) -> EdgeList:
    lib = _load()
    null = ctypes.POINTER(ctypes.c_int32)()
    m = lib.gg_grid(rows, cols, p_keep, p_diag, wmax, seed, null, null,
                    ctypes.POINTER(ctypes.c_uint32)())
    if m < 0:
        raise ValueError("gg_grid: bad arguments")
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    w = np.empty(m, np.uint32)
    m2 = lib.gg_grid(rows, cols, p_keep, p_diag, wmax, seed, _p(src, ctypes.c_int32),
                     _p(dst, ctypes.c_int32), _p(w, ctypes.c_uint32))
    assert m2 == m
    return EdgeList(rows * cols, src, dst, w)


def from_arrays(n: int, src, dst, w) -> EdgeList:
    return EdgeList(int(n), np.ascontiguousarray(src, np.int32), np.ascontiguousarray(dst, np.int32),
                    np.ascontiguousarray(w, np.uint32))


def to_csr(el: EdgeList) -> CSR:
    lib = _load()
    src = np.ascontiguousarray(el.src, np.int32)
    dst = np.ascontiguousarray(el.dst, np.int32)
    w = np.ascontiguousarray(el.w, np.uint32)
    nnz = ctypes.c_int64(0)
    h = lib.gg_csr_build(el.n, src.shape[0], _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32),
                         _p(w, ctypes.c_uint32), ctypes.byref(nnz))
    if not h:
        raise ValueError("gg_csr_build failed (%d)" % nnz.value)
    try:
        rowptr = np.empty(el.n + 1, np.int32)
        col = np.empty(nnz.value, np.int32)
        wo = np.empty(nnz.value, np.uint32)
        lib.gg_csr_copy(h, _p(rowptr, ctypes.c_int32), _p(col, ctypes.c_int32),
                        _p(wo, ctypes.c_uint32))
    finally:
        lib.gg_csr_free(h)
    return CSR(el.n, rowptr, col, wo)


def pick_sources(csr: CSR, k: int, seed: int) -> np.ndarray:
    lib = _load()
    rowptr = np.ascontiguousarray(csr.rowptr, np.int32)
    out = np.empty(max(k, 1), np.int32)
    got = lib.gg_pick_sources(csr.n, _p(rowptr, ctypes.c_int32), k, seed, _p(out, ctypes.c_int32))
    return out[:got].copy()


def permutation(n: int, seed: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, np.int32)
    lib.gg_permutation(n, seed, _p(out, ctypes.c_int32))
    return out


# ---------------------------------------------------------------------------
# Named workloads (shapes of the paper's Section 4.2 graphs; sizes as stated).
# Each returns (EdgeList, CSR).

@dataclasses.dataclass
class Workload:
    name: str
    edges: EdgeList
    csr: CSR
    seed: int

    def sources(self, k: int) -> np.ndarray:
        return pick_sources(self.csr, k, self.seed + 7919)


def binary32_weights(name: str) -> bool:
    """True for the workloads whose weights are binary32 bit patterns
    (rmat<k>f, rmat<k>c<d>)."""
    return name.startswith("rmat") and (name.endswith("f") or "c" in name[4:])


def weight_label(name: str) -> str:
    """The weight distribution of a named workload, as reported."""
    if binary32_weights(name):
        if name.endswith("f"):
            return "binary32, uniform on (0, 1]"
        return "binary32, converge(x, %s) (Eq. 8)" % (int(name.split("c")[1]) / 10.0)
    if name.startswith("rmat") and "p" in name[4:]:
        p = int(name[4:].split("p")[1])
        return "Eq. 7, power %d: 1..%d" % (p, (1 << p) - 1)
    if name.startswith("grid"):
        body = name[4:]
        return "U{1..%s}" % (body.split("w")[1] if "w" in body else "1000")
    return "U{1..255}"


def workload(name: str, scale: Optional[int] = None) -> Workload:
    """Named synthetic workloads.

    ``rmat14``  R-MAT scale 14, edge factor 16, (a,b,c)=(0.57,0.19,0.19), w in 1..255
    ``er22``    G(n, m) with n = 2^22, m = 16 n (mean degree 32), w in 1..255
    ``rmat24``  R-MAT scale 24, edge factor 16, w in 1..255
    ``grid2048`` 2048 x 2048 grid, 5% of edges dropped, 1% diagonals, w in 1..1000
    ``rmat<k>`` / ``er<k>`` / ``grid<k>`` the same recipes at other sizes
    ``grid<k>w<W>``  the grid recipe with w in 1..W (W above 65536: beyond the
                 exact selection-threshold window)
    ``rmat<k>f``  the R-MAT graph rmat<k> with real weights uniform on (0, 1] (binary32 bits)
    ``rmat<k>c<d>``  the same with the float-pivot variant's weights (Eq. 8), pivot d / 10
    ``rmat<k>p<power>``  the R-MAT graph rmat<k> with its weights replaced by the
                 integer-power variant's (Eq. 7): 2^power - 1 distinct weights
    """
    if binary32_weights(name):
        # rmat<k>f: real weights uniform on (0, 1]; rmat<k>c<d>: the float-pivot
        # variant (Eq. 8) with pivot d / 10 -- binary32 bit patterns
        body = name[4:]
        if body.endswith("f"):
            sk, pivot = body[:-1], None
        else:
            sk, d = body.split("c")
            pivot = int(d) / 10.0
        s = int(sk) if scale is None else scale
        seed = SEED_BASE + {14: 1, 24: 3, 22: 5}.get(s, 100 + s)
        el = rmat(s, 16, 0.57, 0.19, 0.19, 255, seed)
        el = EdgeList(el.n, el.src, el.dst, weights_f32(el.src.shape[0], seed, pivot))
    elif name.startswith("rmat") and "p" in name[4:]:
        sk, pw = name[4:].split("p")
        s = int(sk) if scale is None else scale
        seed = SEED_BASE + {14: 1, 24: 3, 22: 5}.get(s, 100 + s)
        el = rmat(s, 16, 0.57, 0.19, 0.19, 255, seed)
        el = EdgeList(el.n, el.src, el.dst, weights_power(el.src.shape[0], int(pw), seed))
    elif name.startswith("rmat"):
        s = int(name[4:]) if scale is None else scale
        seed = SEED_BASE + {14: 1, 24: 3, 22: 5}.get(s, 100 + s)
        el = rmat(s, 16, 0.57, 0.19, 0.19, 255, seed)
    elif name.startswith("er"):
        s = int(name[2:]) if scale is None else scale
        seed = SEED_BASE + {22: 2}.get(s, 200 + s)
        n = 1 << s
        el = gnm(n, 16 * n, 255, seed)
    elif name.startswith("grid"):
        # grid<side>, or grid<side>w<W>: the same recipe with w in 1..W
        body = name[4:]
        sk, wk = body.split("w") if "w" in body else (body, "1000")
        side = int(sk) if scale is None else scale
        seed = SEED_BASE + {2048: 4}.get(side, 300 + side)
        el = grid(side, side, 0.95, 0.01, int(wk), seed)
    else:
        raise ValueError("unknown workload %r" % name)
    return Workload(name, el, to_csr(el), seed)


def small_rmat_batch(count: int = 256, lo: int = 10, hi: int = 16) -> list:
    """The batch of small graphs: `count` R-MAT graphs (edge factor 16, the same
    (a, b, c), w in 1..255) with scales drawn uniformly from lo..hi, one source
    each. Returns a list of Workload."""
    rng = np.random.default_rng(SEED_BASE + 6)
    scales = rng.integers(lo, hi + 1, size=count)
    out = []
    for i, sc in enumerate(scales):
        seed = SEED_BASE + 1000 + i
        el = rmat(int(sc), 16, 0.57, 0.19, 0.19, 255, seed)
        out.append(Workload("rmat%d_b%d" % (int(sc), i), el, to_csr(el), seed))
    return out


def poisson_trace(count: int, rate: float, n_graphs: int, seed: int = SEED_BASE + 7) -> tuple:
    """A query trace: arrival times (seconds, Poisson process of the given
    rate) and the graph index of each query (uniform over n_graphs)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    which = rng.integers(0, n_graphs, size=count)
    return arrivals, which
