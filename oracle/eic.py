"""ORACLE -- test infrastructure only; the product path never imports this.

A sequential model of the paper's heuristic SSSP method (Section 3), used to
pin the GPU engine's schedule. It is built from the method's definitions:

* the band <lb, ub> of a step is settled to a fixpoint by synchronous
  relaxation rounds restricted to the band (Section 3.3); during the first
  step ub follows the nearest vertex of degree >= highD(0);
* before the rounds, vertices already settled in [lb0, st] relax the edges
  they had to defer (their sums now fall in the band), and, when the
  selection threshold st lies below lb, every unsettled vertex takes its best
  neighbour settled in [st, lb) whose sum lands in the band (the pull of
  Section 3.2);
* after the band is settled, the statistics at L = ub (sumD, highD) give
  gap(L) (Eq. 1-3), the next band is <L, L + gap(L)>, and st for it comes
  from computeST (Eq. 4-6);
* the search ends when no remaining distance can still fall below the band.

Every relaxation of a round reads the distances the round started with, and
the round's candidates are merged with a minimum (any order reaches the same
fixpoint). The model serves two purposes in the tests: it must reach exactly
the Dijkstra distances (the heuristics only reorder relaxations), and its
per-step schedule -- <lb, ub, st> and the statistics taken at each step's end
-- is determined by the graph and the source alone (every quantity used at a
step boundary is a function of the settled set, whose distances are final),
so the GPU engine has to produce the same schedule step for step.

Distances are integers (uint32 range, +inf = 2^32 - 1, sums exact in int64)
or binary32 bit patterns (finite, non-negative, so they order like their
values; every sum is one binary32 addition rounded to nearest). The two
differ only in how distances add, how the band's ends and lb0 are formed and
which computeST runs; `_Integers` and `_Binary32` hold those rules.

Readings of the text it follows: the first step's hub update of ub runs only
during the first step; the first step ends the search when no vertex of
degree >= highD(0) was reached (ub stays +inf); the v != parent[u] skip is
omitted (no parent[] is produced).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

from . import heuristic as H

INF = H.INF


@dataclasses.dataclass
class Step:
    lb: int          # band of this step
    ub: int
    st: int          # selection threshold used by this step
    rounds: int      # push rounds of this step
    pulled: bool     # whether the pull ran (st < lb)
    L: int           # next threshold (= this step's final ub)
    S: int           # sumD(L)
    h: int           # highD(L)
    gap: int         # gap(L)
    st_next: int     # computeST for <L, L + gap(L)>


@dataclasses.dataclass
class Result:
    dist: np.ndarray
    steps: List[Step]
    expansions: int = 0
    band_expansions: int = 0
    push_scanned: int = 0
    pull_vertices: int = 0
    pull_scanned: int = 0
    rounds: int = 0
    pulls: int = 0
    high_d0: int = 0
    gap0: int = 0
    complete: bool = True   # False: max_steps ended the model before its stopping test


def _row_edges(rowptr: np.ndarray, rows: np.ndarray) -> tuple:
    """Edge indices of the given rows, and the row each index belongs to."""
    starts = rowptr[rows].astype(np.int64)
    lens = (rowptr[rows + 1] - rowptr[rows]).astype(np.int64)
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    owner = np.repeat(np.arange(rows.shape[0]), lens)
    first = np.cumsum(lens) - lens
    idx = starts[owner] + (np.arange(total) - first[owner])
    return idx, rows[owner]


def _fadd(a, b) -> np.ndarray:
    """fl(a + b) of binary32 bit patterns, elementwise, as bit patterns (int64)."""
    a = np.asarray(a, dtype=np.int64).astype(np.uint32).view(np.float32)
    b = np.asarray(b, dtype=np.int64).astype(np.uint32).view(np.float32)
    return (a + b).astype(np.float32).view(np.uint32).astype(np.int64)


# ---------------------------------------------------------- distance rules --

class _Integers:
    """Integer weights: exact sums. computeST scores the exact window of
    distinct settled distances while maxW <= ST_NUM, where a bin of Section
    4.1's grid (ST_NUM per maxW) is at most one distance unit wide, and the
    grid above (st_grid None); st_grid True asks for the grid always, False
    for the window while it fits (maxW <= ST_WINDOW_MAX)."""

    inf = INF

    def __init__(self, w: np.ndarray, st_grid=None):
        self.w = np.asarray(w, dtype=np.int64)
        M = int(self.w.max()) if self.w.shape[0] else 0
        if M > H.ST_WINDOW_MAX:
            self.grid = True
        elif st_grid is None:
            self.grid = M > H.ST_NUM
        else:
            self.grid = bool(st_grid)

    def add(self, d, w):
        return d + w

    def reaches_below(self, st: int, w: np.ndarray, ub: int) -> np.ndarray:
        # the pull takes an edge of weight w while w < ub - st (Section 3.2)
        return w < ub - st

    def low_end(self, lb: int, M: int) -> int:
        # lb0 = max(0, lb - M): the settled vertices whose deferred edges can
        # land in the band
        return max(0, lb - M)

    def band_end(self, L: int, gap: int) -> int:
        return min(L + gap, INF)

    def threshold(self, dist, deg, L, gap_L, gap_lb, S, nnz, M, lb0, ub_next, traversal_opt) -> int:
        win = (dist >= lb0) & (dist < L)
        vals, inv = np.unique(dist[win], return_inverse=True)
        mass = np.zeros(vals.shape[0], dtype=np.int64)
        np.add.at(mass, inv, deg[win])
        if self.grid:
            return H.compute_st_grid(L, gap_L, gap_lb, S, nnz, M, lb0, ub_next, vals, mass, False,
                                     traversal_opt)
        return H.compute_st(L, gap_L, gap_lb, S, nnz, M, vals, mass, traversal_opt)

    def stop_at_infinite_band(self) -> bool:
        return False

    def beyond(self, dmax: int, M: int, lb: int) -> bool:
        return dmax + M < lb


class _Binary32:
    """Binary32 weights and distances (bit patterns): each sum rounds once;
    computeST always scores the ST_NUM grid."""

    inf = INF   # the shared +inf sentinel; finite bit patterns stay below 0x7f800000

    def __init__(self, w: np.ndarray):
        self.w = np.asarray(w, dtype=np.uint32).astype(np.int64)
        pos = self.w[self.w > 0]
        self.minpos = int(pos.min()) if pos.shape[0] else INF

    def add(self, d, w):
        return _fadd(d, w)

    def reaches_below(self, st: int, w: np.ndarray, ub: int) -> np.ndarray:
        # w < ub - st, rounded: a settled distance d >= st reaches below ub
        # only if fl(st + w) does (rounding is monotone)
        return _fadd(np.full(w.shape[0], st), w) < ub

    def low_end(self, lb: int, M: int) -> int:
        # lb - M lowered by two units in the last place of lb, so that a settled
        # distance whose rounded sum with M still reaches lb is included
        if lb == 0:
            return 0
        Lf = np.float32(H.f32(lb))
        ulp = np.float32(H.f32(lb + 1)) - Lf
        lo = np.float32(np.float32(Lf - np.float32(H.f32(M))) - np.float32(np.float32(2.0) * ulp))
        return int(np.asarray(lo, dtype=np.float32).view(np.uint32)) if lo > 0 else 0

    def band_end(self, L: int, gap: int) -> int:
        # ub = L + gap(L) (Section 3.3), rounded. The gap is positive (Section
        # 3.1 keeps it in (0, maxW]): a zero quantile takes the smallest
        # positive weight; and the next band ends above L even where the sum
        # rounds back to L
        g = gap if (gap > self.minpos or self.minpos == INF) else self.minpos
        e = int(_fadd(L, g))
        if e <= L:
            e = L + 1
        return INF if e >= H.F32_INF_BITS else e

    def threshold(self, dist, deg, L, gap_L, gap_lb, S, nnz, M, lb0, ub_next, traversal_opt) -> int:
        settled = dist < L
        return H.compute_st_f32(L, gap_L, gap_lb, S, nnz, M, lb0, ub_next, dist[settled], deg[settled],
                                traversal_opt)

    def stop_at_infinite_band(self) -> bool:
        return True

    def beyond(self, dmax: int, M: int, lb: int) -> bool:
        return int(_fadd(dmax, M)) < lb


# ------------------------------------------------------------ step pieces --

class _Search:
    """One search: the graph, the distance rules and the running state."""

    def __init__(self, n, rowptr, col, rules, s):
        self.n = n
        self.rowptr = np.asarray(rowptr, dtype=np.int64)
        self.col = np.asarray(col, dtype=np.int64)
        self.rules = rules
        self.w = rules.w
        self.deg = np.diff(self.rowptr)
        self.nnz = int(self.rowptr[-1])
        self.M = int(self.w.max()) if self.nnz else 0
        # Section 4.1's preprocessing: the weight quantiles and highD over VS(0) = V
        self.rtow = H.rtow_table(self.w)
        self.hd0 = H.high_d(self.deg)
        self.hub = self.deg >= max(self.hd0, 1)
        self.dist = np.full(n, INF, dtype=np.int64)
        self.dist[s] = 0
        self.res = Result(dist=self.dist, steps=[], high_d0=self.hd0)

    def deferred(self, lb0: int, st: int) -> np.ndarray:
        """Settled vertices in [lb0, st]: their edges deferred past earlier bands."""
        d = self.dist
        return np.nonzero((d >= lb0) & (d <= st))[0]

    def pull(self, st: int, lb: int, ub: int) -> None:
        """Every unsettled vertex of degree >= 1 takes its best neighbour settled
        in [st, lb) through an edge short enough to land in the band."""
        d, res = self.dist, self.res
        res.pulls += 1
        unsettled = np.nonzero((d > lb) & (self.deg > 0))[0]
        res.pull_vertices += int(unsettled.shape[0])
        idx, owner = _row_edges(self.rowptr, unsettled)
        keep = self.rules.reaches_below(st, self.w[idx], ub)
        idx, owner = idx[keep], owner[keep]
        res.pull_scanned += int(idx.shape[0])
        dv = d[self.col[idx]]
        ok = (dv >= st) & (dv < lb)
        cand = self.rules.add(np.where(ok, dv, 0), self.w[idx])
        ok &= cand < ub
        np.minimum.at(d, owner[ok], cand[ok])

    def settle_band(self, frontier: np.ndarray, lb: int, ub: int, first: bool) -> tuple:
        """Synchronous relaxation rounds restricted to the band until no
        distance changes; leaves (degree 1, not the source) are not expanded.
        In the first step ub follows the nearest hub after every round.
        Returns (rounds, ub)."""
        d, res = self.dist, self.res
        rounds = 0
        while frontier.shape[0] > 0:
            paths = frontier[~((d[frontier] > 0) & (self.deg[frontier] == 1))]
            res.expansions += int(paths.shape[0])
            res.band_expansions += int(np.count_nonzero(d[paths] >= lb))
            idx, owner = _row_edges(self.rowptr, paths)
            cand = self.rules.add(d[owner], self.w[idx])
            inside = (cand >= lb) & (cand < ub)
            idx, cand = idx[inside], cand[inside]
            res.push_scanned += int(idx.shape[0])
            before = d.copy()
            np.minimum.at(d, self.col[idx], cand)
            frontier = np.nonzero(d < before)[0]
            rounds += 1
            if first:
                hub_d = d[self.hub]
                ub = int(hub_d.min()) if hub_d.shape[0] else INF
        res.rounds += rounds
        return rounds, ub

    def statistics(self, L: int, alpha: int, beta: float) -> tuple:
        """sumD(L) and highD(L) over VS(L) = {v : dist[v] >= L}, and gap(L) (Eq. 1-3)."""
        in_vs = self.dist >= L
        S = int(self.deg[in_vs].sum())
        h = H.high_d(self.deg[in_vs])
        return S, h, H.gap(S, h, self.nnz, self.M, self.rtow, alpha, beta)


def _model(n, rowptr, col, rules, s, alpha, beta, traversal_opt, max_steps) -> Result:
    run = _Search(n, rowptr, col, rules, s)
    res, dist, M = run.res, run.dist, run.M
    if run.deg[s] == 0:
        res.dist = dist.astype(np.uint32)
        return res
    res.gap0 = H.gap(run.nnz, run.hd0, run.nnz, M, run.rtow, alpha, beta)
    st, lb, ub = 0, 0, INF
    first = True
    gap_lb = res.gap0   # gap of the band just settled (gap(0) before the first)
    for _ in range(max_steps):
        frontier = run.deferred(rules.low_end(lb, M), st)
        pulled = st < lb
        if pulled:
            run.pull(st, lb, ub)
        band = np.nonzero((dist >= lb) & (dist < ub))[0]
        rounds, ub = run.settle_band(np.union1d(frontier, band), lb, ub, first)
        if first and ub == INF:
            # no hub reached: the first band was the whole reachable set
            res.steps.append(Step(lb, ub, st, rounds, pulled, ub, 0, 0, 0, ub))
            break
        L = ub
        S, h, gap_L = run.statistics(L, alpha, beta)
        if L == INF and rules.stop_at_infinite_band():
            res.steps.append(Step(lb, ub, st, rounds, pulled, L, S, h, gap_L, L))
            break
        ub_next = rules.band_end(L, gap_L)
        st_next = rules.threshold(dist, run.deg, L, gap_L, gap_lb, S, run.nnz, M, rules.low_end(L, M),
                                  ub_next, traversal_opt)
        res.steps.append(Step(lb, ub, st, rounds, pulled, L, S, h, gap_L, st_next))
        st, lb, ub = st_next, L, ub_next
        gap_lb = gap_L
        first = False
        if rules.beyond(int(dist[dist < INF].max()), M, lb):
            break
    else:
        res.complete = False
    res.dist = dist.astype(np.uint32)
    return res


def eic_sssp(n: int, rowptr: np.ndarray, col: np.ndarray, w: np.ndarray, s: int,
             alpha: int = H.ALPHA, beta: float = H.BETA, traversal_opt: bool = True,
             max_steps: int = 10_000_000, st_grid=None) -> Result:
    """The model with integer weights; st_grid: computeST's candidates (None:
    the exact window while maxW <= ST_NUM, the ST_NUM grid above; True: the
    grid; False: the window while maxW <= 65536)."""
    return _model(n, rowptr, col, _Integers(w, st_grid), s, alpha, beta, traversal_opt, max_steps)


def eic_sssp_f32(n: int, rowptr: np.ndarray, col: np.ndarray, wbits: np.ndarray, s: int,
                 alpha: int = H.ALPHA, beta: float = H.BETA, traversal_opt: bool = True,
                 max_steps: int = 10_000_000) -> Result:
    """The model with real weights: weights and distances are binary32 bit
    patterns. A band narrower than the spacing of the remaining distances
    settles nothing and the next one starts where it ended, as with integers
    and gap 1: weights that span many orders of magnitude (say 1e-30 and 1e30
    in one graph) can need a step per unit in the last place. `complete` is
    False when max_steps ran out first."""
    return _model(n, rowptr, col, _Binary32(wbits), s, alpha, beta, traversal_opt, max_steps)


def normalised(res: Result, n: int, deg: np.ndarray) -> dict:
    """The paper's normalised counters (Section 4): nFrontier over reachable
    non-leaf vertices, nSync over log2|V|, nTrav over reachable vertices.
    nFrontier counts the extended paths of the band (vertices at or above lb
    when expanded); nExpand also counts the settled vertices re-expanded for
    their deferred long edges."""
    deg = np.asarray(deg)
    reach = res.dist != np.uint32(INF)
    n_reach = int(reach.sum())
    nonleaf = int((reach & (deg > 1)).sum()) or 1
    syncs = res.rounds + res.pulls
    return {
        "nFrontier": res.band_expansions / nonleaf,
        "nExpand": res.expansions / nonleaf,
        "nSync": syncs / math.log2(max(n, 2)),
        "nTrav": (res.push_scanned + res.pull_scanned) / max(n_reach, 1),
        "steps": len(res.steps),
        "syncs": syncs,
    }
