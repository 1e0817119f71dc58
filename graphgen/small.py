"""Small seeded graphs for exhaustive and closed-form tests (inputs only)."""
from __future__ import annotations

import numpy as np

from . import EdgeList, from_arrays


def tiny_random(n: int, m: int, weights, seed: int, self_loops: bool = True) -> EdgeList:
    """m undirected edges with uniform endpoints (parallel edges and, if
    allowed, self-loops included); weights drawn uniformly from `weights`."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    w = rng.choice(np.asarray(weights, dtype=np.uint64), size=src.shape[0])
    return from_arrays(n, src, dst, w)


def path(n: int, weights) -> EdgeList:
    """0-1-2-...-(n-1) with weights[i] on edge (i, i+1)."""
    src = np.arange(n - 1)
    return from_arrays(n, src, src + 1, np.asarray(weights, dtype=np.uint64)[: n - 1])


def lattice(rows: int, cols: int, c: int) -> EdgeList:
    """Full 4-neighbour lattice, every edge of weight c; vertex r*cols + k."""
    ids = np.arange(rows * cols).reshape(rows, cols)
    s = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    d = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_arrays(rows * cols, s, d, np.full(s.shape[0], c, dtype=np.uint64))


def star(leaves: int, weights) -> EdgeList:
    """Hub 0 joined to vertices 1..leaves."""
    d = np.arange(1, leaves + 1)
    return from_arrays(leaves + 1, np.zeros(leaves, dtype=np.int64), d,
                       np.asarray(weights, dtype=np.uint64)[:leaves])


def disjoint_union(a: EdgeList, b: EdgeList) -> EdgeList:
    return from_arrays(a.n + b.n, np.concatenate([a.src, b.src + a.n]),
                       np.concatenate([a.dst, b.dst + a.n]), np.concatenate([a.w, b.w]))
