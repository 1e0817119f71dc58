"""ORACLE -- test infrastructure only; the product path never imports this.

A sequential model of the paper's heuristic SSSP algorithm (Section 3.3: the
Algorithm, Function 1 initFrontiers and Function 2 computeST), written in the
paper's order and notation with numpy doing the per-round vector work.
Rounds are synchronous: every relaxation of a round reads the distances the
round started with, and the round's candidates are merged with a minimum.

It serves two purposes in the tests:
* it must reach exactly the Dijkstra distances (the method is exact: the
  heuristics only reorder relaxations), and
* its per-step schedule -- the band <lb, ub>, the selection threshold st and
  the statistics taken at each step's end -- is fully determined by the graph
  and the source (every quantity it uses at a step boundary is a function of
  the settled set, whose distances are final), so the GPU engine has to
  produce the same schedule step for step.

Readings of the text it follows: the first step's
hub update of ub runs only during the first step; the first step ends the
search when no vertex of degree >= highD(0) was reached (ub stays +inf);
+inf is the single sentinel 2^32 - 1; the v != parent[u] skip is omitted
(no parent[] is produced).
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


def eic_sssp(n: int, rowptr: np.ndarray, col: np.ndarray, w: np.ndarray, s: int,
             alpha: int = H.ALPHA, beta: float = H.BETA, traversal_opt: bool = True,
             max_steps: int = 10_000_000) -> Result:
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    deg = np.diff(rowptr)
    nnz = int(rowptr[-1])
    M = int(w.max()) if nnz else 0
    # Preprocess (Section 4.1): weight quantisation; highD(0) over VS(0) = V.
    rtow = H.rtow_table(w)
    hd0 = H.high_d(deg)
    hub = (deg >= max(hd0, 1))

    dist = np.full(n, INF, dtype=np.int64)
    dist[s] = 0
    res = Result(dist=dist, steps=[], high_d0=hd0)
    if deg[s] == 0:
        res.dist = dist.astype(np.uint32)
        return res
    res.gap0 = H.gap(nnz, hd0, nnz, M, rtow, alpha, beta)

    st, lb, ub = 0, 0, INF
    first = True
    gap_lb = res.gap0
    for _ in range(max_steps):
        # ---- Function 1: initFrontiers(st, lb, ub) ----
        lb0 = max(0, lb - M)
        push_set = np.nonzero((dist >= lb0) & (dist <= st))[0]
        pulled = False
        if st < lb:
            pulled = True
            res.pulls += 1
            U = np.nonzero((dist > lb) & (deg > 0))[0]
            res.pull_vertices += int(U.shape[0])
            idx, owner = _row_edges(rowptr, U)
            sel = w[idx] < ub - st
            idx, owner = idx[sel], owner[sel]
            res.pull_scanned += int(idx.shape[0])
            v = col[idx]
            dv = dist[v]
            cand = dv + w[idx]
            ok = (dv >= st) & (dv < lb) & (cand < ub)
            np.minimum.at(dist, owner[ok], cand[ok])
        band = np.nonzero((dist >= lb) & (dist < ub))[0]
        F = np.union1d(push_set, band)
        rounds = 0
        # ---- the Algorithm's round loop ----
        while F.shape[0] > 0:
            paths = F[~((dist[F] > 0) & (deg[F] == 1))]
            res.expansions += int(paths.shape[0])
            res.band_expansions += int(np.count_nonzero(dist[paths] >= lb))
            idx, owner = _row_edges(rowptr, paths)
            cand = dist[owner] + w[idx]
            sel = (cand >= lb) & (cand < ub)
            idx, cand = idx[sel], cand[sel]
            res.push_scanned += int(idx.shape[0])
            v = col[idx]
            before = dist.copy()
            np.minimum.at(dist, v, cand)
            F = np.nonzero(dist < before)[0]
            rounds += 1
            if first:
                hub_d = dist[hub]
                ub = int(hub_d.min()) if hub_d.shape[0] else INF
        res.rounds += rounds
        if first and ub == INF:
            res.steps.append(Step(lb, ub, st, rounds, pulled, ub, 0, 0, 0, ub))
            break
        # ---- statistics at L = ub, then <st, lb, ub> <- <computeST, ub, ub + gap(ub)> ----
        L = ub
        in_vs = dist >= L
        S = int(deg[in_vs].sum())
        h = H.high_d(deg[in_vs])
        gap_L = H.gap(S, h, nnz, M, rtow, alpha, beta)
        wlo = max(0, L - M)
        win = (dist >= wlo) & (dist < L)
        wv, inv = np.unique(dist[win], return_inverse=True)
        wm = np.zeros(wv.shape[0], dtype=np.int64)
        np.add.at(wm, inv, deg[win])
        st_next = H.compute_st(L, gap_L, gap_lb, S, nnz, M, wv, wm, traversal_opt)
        res.steps.append(Step(lb, ub, st, rounds, pulled, L, S, h, gap_L, st_next))
        st, lb, ub = st_next, L, min(L + gap_L, INF)
        gap_lb = gap_L
        first = False
        finite = dist[dist < INF]
        if int(finite.max()) + M < lb:
            break
    else:
        res.complete = False
    res.dist = dist.astype(np.uint32)
    return res


def _fadd(a, b) -> np.ndarray:
    """fl(a + b) of binary32 bit patterns, elementwise, as bit patterns (int64)."""
    a = np.asarray(a, dtype=np.int64).astype(np.uint32).view(np.float32)
    b = np.asarray(b, dtype=np.int64).astype(np.uint32).view(np.float32)
    return (a + b).astype(np.float32).view(np.uint32).astype(np.int64)


def eic_sssp_f32(n: int, rowptr: np.ndarray, col: np.ndarray, wbits: np.ndarray, s: int,
                 alpha: int = H.ALPHA, beta: float = H.BETA, traversal_opt: bool = True,
                 max_steps: int = 10_000_000) -> Result:
    """The same model with real weights: weights and distances are binary32
    bit patterns (finite, non-negative, so they order like their values) and
    every path sum is one binary32 addition, rounded to nearest.  The readings
    that differ from the integer model: the next band ends at fl(L + gap)
    with the gap at least the smallest positive weight, and one unit in the
    last place above L when that sum rounds back to L (ub > lb, Section 3);
    lb0 = fl(fl(L - M) - 2 ulp(L)); the pull takes an edge while
    fl(st + w) < ub; computeST works on the ST_NUM grid.

    A band narrower than the spacing of the remaining distances settles
    nothing and the next one starts where it ended, as in the integer model:
    weights that span many orders of magnitude (say 1e-30 and 1e30 in one
    graph) can need a step per unit in the last place. `complete` is False
    when max_steps ran out first."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    w = np.asarray(wbits, dtype=np.uint32).astype(np.int64)
    deg = np.diff(rowptr)
    nnz = int(rowptr[-1])
    M = int(w.max()) if nnz else 0
    pos = w[w > 0]
    minpos = int(pos.min()) if pos.shape[0] else INF
    rtow = H.rtow_table(w)
    hd0 = H.high_d(deg)
    hub = (deg >= max(hd0, 1))

    dist = np.full(n, INF, dtype=np.int64)
    dist[s] = 0
    res = Result(dist=dist, steps=[], high_d0=hd0)
    if deg[s] == 0:
        res.dist = dist.astype(np.uint32)
        return res
    res.gap0 = H.gap(nnz, hd0, nnz, M, rtow, alpha, beta)

    st, lb, ub, lb0 = 0, 0, INF, 0
    first = True
    gap_lb = res.gap0
    for _ in range(max_steps):
        # ---- Function 1: initFrontiers(st, lb, ub) ----
        push_set = np.nonzero((dist >= lb0) & (dist <= st))[0]
        pulled = False
        if st < lb:
            pulled = True
            res.pulls += 1
            U = np.nonzero((dist > lb) & (deg > 0))[0]
            res.pull_vertices += int(U.shape[0])
            idx, owner = _row_edges(rowptr, U)
            sel = _fadd(np.full(idx.shape[0], st), w[idx]) < ub
            idx, owner = idx[sel], owner[sel]
            res.pull_scanned += int(idx.shape[0])
            dv = dist[col[idx]]
            ok = (dv >= st) & (dv < lb)
            cand = _fadd(np.where(ok, dv, 0), w[idx])
            ok &= cand < ub
            np.minimum.at(dist, owner[ok], cand[ok])
        band = np.nonzero((dist >= lb) & (dist < ub))[0]
        F = np.union1d(push_set, band)
        rounds = 0
        # ---- the Algorithm's round loop ----
        while F.shape[0] > 0:
            paths = F[~((dist[F] > 0) & (deg[F] == 1))]
            res.expansions += int(paths.shape[0])
            res.band_expansions += int(np.count_nonzero(dist[paths] >= lb))
            idx, owner = _row_edges(rowptr, paths)
            cand = _fadd(dist[owner], w[idx])
            sel = (cand >= lb) & (cand < ub)
            idx, cand = idx[sel], cand[sel]
            res.push_scanned += int(idx.shape[0])
            before = dist.copy()
            np.minimum.at(dist, col[idx], cand)
            F = np.nonzero(dist < before)[0]
            rounds += 1
            if first:
                hub_d = dist[hub]
                ub = int(hub_d.min()) if hub_d.shape[0] else INF
        res.rounds += rounds
        if first and ub == INF:
            res.steps.append(Step(lb, ub, st, rounds, pulled, ub, 0, 0, 0, ub))
            break
        # ---- statistics at L = ub; the next band, lb0 and computeST ----
        L = ub
        in_vs = dist >= L
        S = int(deg[in_vs].sum())
        h = H.high_d(deg[in_vs])
        gap_L = H.gap(S, h, nnz, M, rtow, alpha, beta)
        if L == INF:
            res.steps.append(Step(lb, ub, st, rounds, pulled, L, S, h, gap_L, L))
            break
        # ub = L + gap(L) (Section 3.3), rounded; the gap is positive (Section
        # 3.1: gap in (0, maxW]), so a zero quantile takes the smallest positive
        # weight, and ub > lb holds even where the sum rounds back to L
        gf = gap_L if (gap_L > minpos or minpos == INF) else minpos
        e = int(_fadd(L, gf))
        if e <= L:
            e = L + 1
        ub_next = INF if e >= H.F32_INF_BITS else e
        Lf = np.float32(H.f32(L))
        ulp = np.float32(H.f32(L + 1)) - Lf
        lo = np.float32(np.float32(Lf - np.float32(H.f32(M))) - np.float32(np.float32(2.0) * ulp))
        lb0_next = int(np.asarray(lo, dtype=np.float32).view(np.uint32)) if lo > 0 else 0
        settled = dist < L
        st_next = H.compute_st_f32(L, gap_L, gap_lb, S, nnz, M, lb0_next, ub_next, dist[settled],
                                   deg[settled], traversal_opt)
        res.steps.append(Step(lb, ub, st, rounds, pulled, L, S, h, gap_L, st_next))
        st, lb, ub, lb0 = st_next, L, ub_next, lb0_next
        gap_lb = gap_L
        first = False
        finite = dist[dist < INF]
        if int(_fadd(int(finite.max()), M)) < lb:
            break
    else:
        res.complete = False
    res.dist = dist.astype(np.uint32)
    return res


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
