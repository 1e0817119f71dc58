"""ORACLE -- test infrastructure only; the product path never imports this.

The statistics and the two heuristics of the paper's Section 3, restated from
the text in plain numpy / Python arithmetic:

* the graph statistics sumD, highD and maxW (Section 3, list of statistics),
* the RtoW[] weight quantisation (Section 4.1),
* dynamic stepping: prob, ratio and gap, Eq. (1)-(3) (Section 3.1),
* traversal optimisation: pushed, pulled and long, Eq. (4)-(6), with the
  lb_0 / ub_0 / ub_1 clamps of Section 3.2, and Function 2 (computeST).

Readings where the text is silent or ambiguous:

* |E| is the undirected edge count, so 2|E| = nnz, the number of CSR entries
  (the sum of all degrees); "sumD >= |E|" is tested as 2*sumD >= nnz.
* highD: candidate thresholds are the distinct degrees >= 1 present in VS; the
  low set is deg < h, the high set deg >= h; ties go to the smallest h; an empty
  VS (or one with no degree mass) gives h = 0.
* maxW(G, r) is the r-quantile of the nnz CSR weights: the smallest weight w
  such that at least ceil(r * nnz) entries are <= w.  RtoW[x] = maxW(G,
  x / (RATIO_NUM - 1)); gap looks up RtoW[ceil(ratio * (RATIO_NUM - 1))].
* gap is at least 1 (integer weights may make the quantile 0).
* computeST is evaluated for the NEXT pair <L, L + gap(L)>; its gap(lb) guard
  uses the gap of the step that just ended (gap(0) from whole-graph statistics
  for the first step).  Candidates are the distinct settled distances in
  [max(0, L - M), L) in ascending order; the first strict maximum above 0 wins,
  otherwise L.  Below L - M every candidate clamps to the same estimate.
* Eq. (4)-(6) are evaluated in IEEE double with the operation order written
  here and no fused multiply-add.
* When the largest weight exceeds ST_WINDOW_MAX the exact window of candidate
  distances is not kept: computeST scores the points of the ST_NUM grid
  instead, as for real weights (below). (The schedule model scores the grid by
  default once the largest weight exceeds ST_NUM, where the window would hold
  more candidates than the grid.)
* A single sentinel INF = 2^32 - 1 stands for +infinity in dist, ub and every
  threshold; sums are clamped to it.
* The ST_NUM grid (real binary32 weights, and integer weights beyond the
  exact window): ST_NUM (Section 4.1: 2^10) equal bins per maxW, bin(d) =
  floor(d * ST_NUM / maxW) in double; a candidate is a grid point whose bin
  holds a settled vertex and has no distance below lb0 = L - M (for binary32,
  lowered by two units in the last place of L), scored by Eq. 4-6 at the grid
  point, and the threshold returned is the smallest distance (bit pattern, or
  integer) of the winning bin.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA = 3          # Section 4.1 configuration <alpha, beta> = <3, 0.9>
BETA = 0.9
RATIO_NUM = 4096   # Section 4.1: RATIO_NUM = 2^12
INF = 0xFFFFFFFF
ST_WINDOW_MAX = 65536
ST_NUM = 1024      # Section 4.1: ST_NUM = 2^10
F32_INF_BITS = 0x7F800000


def rtow_table(weights: np.ndarray, ratio_num: int = RATIO_NUM) -> np.ndarray:
    """RtoW[x] = maxW(G, x / (ratio_num - 1)) over the CSR weight multiset (Section 4.1)."""
    ws = np.sort(np.asarray(weights, dtype=np.uint64))
    nnz = int(ws.shape[0])
    out = np.zeros(ratio_num, dtype=np.uint32)
    if nnz == 0:
        return out
    for x in range(ratio_num):
        need = -((-x * nnz) // (ratio_num - 1))  # ceil(x * nnz / (ratio_num - 1))
        out[x] = ws[max(need, 1) - 1]
    return out


def max_w(weights: np.ndarray, r: float) -> int:
    """maxW(G, r): the smallest weight w with at least ceil(r * nnz) weights <= w."""
    ws = np.sort(np.asarray(weights, dtype=np.uint64))
    need = math.ceil(r * ws.shape[0])
    return int(ws[max(need, 1) - 1])


def sum_d(deg: np.ndarray, dist: np.ndarray, lb: int) -> int:
    """sumD(lb): total degree of VS(lb) = {x : dist[x] >= lb} (unreached vertices included)."""
    return int(np.asarray(deg, dtype=np.int64)[np.asarray(dist) >= lb].sum())


def high_d(degs_in_vs: np.ndarray) -> int:
    """highD over a vertex set given by its degrees: the threshold h splitting
    the set into {deg < h} and {deg >= h} with the least difference in total
    degree (Section 3, statistics list).  Smallest h on ties; 0 if no mass."""
    d = np.asarray(degs_in_vs, dtype=np.int64)
    d = d[d >= 1]
    if d.shape[0] == 0:
        return 0
    vals, counts = np.unique(d, return_counts=True)
    mass = vals * counts.astype(np.int64)
    total = int(mass.sum())
    low = np.concatenate([[0], np.cumsum(mass)[:-1]])
    diff = np.abs(2 * low - total)
    return int(vals[int(np.argmin(diff))])


def prob(S: int, nnz: int, beta: float = BETA) -> float:
    """Eq. (1): prob = min(beta, max(sumD, 2|E| - sumD) / 2|E|)."""
    return min(beta, max(S, nnz - S) / nnz)


def ratio(p: float, h: int) -> float:
    """Eq. (2): ratio = 1 - (1 - prob)^(1 / (prob * highD))."""
    return 1.0 - (1.0 - p) ** (1.0 / (p * h))


def ratio_index(r: float, ratio_num: int = RATIO_NUM) -> int:
    return min(ratio_num - 1, max(0, math.ceil(r * (ratio_num - 1))))


def gap(S: int, h: int, nnz: int, M: int, rtow: np.ndarray, alpha: int = ALPHA,
        beta: float = BETA) -> int:
    """Eq. (3): gap = maxW(G, 1) if highD <= alpha, else maxW(G, ratio); at least 1."""
    if h <= alpha:
        g = M
    else:
        g = int(rtow[ratio_index(ratio(prob(S, nnz, beta), h))])
    return max(1, g)


def profit(x: int, L: int, Y: int, S: int, Sx: int, M: int, nnz: int) -> float:
    """Eq. (4)-(6) for selection threshold x and the pair <L, Y>, with the
    clamps lb_0 = max(x, L - M), ub_0 = min(Y, L + M), ub_1 = min(Y, lb_0 + M)
    (Section 3.2).  Sx = sumD(lb_0), S = sumD(L)."""
    lb0 = max(x, L - M)
    ub0 = min(Y, L + M)
    ub1 = min(Y, lb0 + M)
    pushed = float(ub0 - L) * float(Sx - S) / float(M)
    pulled = float(ub1 - lb0) * float(S) / float(M)
    long_ = pulled * float(Sx - S) / float(nnz)
    return (pushed - long_) - pulled


def compute_st(L: int, gap_L: int, gap_lb: int, S: int, nnz: int, M: int,
               win_vals: np.ndarray, win_mass: np.ndarray, traversal_opt: bool = True) -> int:
    """Function 2 (computeST) for the next pair <L, L + gap(L)>.

    win_vals: distinct settled distances in [max(0, L - M), L), ascending;
    win_mass: total degree of the settled vertices at each of those distances.
    """
    if traversal_opt and M > ST_WINDOW_MAX:
        # beyond the exact window: the ST_NUM grid
        return compute_st_grid(L, gap_L, gap_lb, S, nnz, M, max(0, L - M), min(L + gap_L, INF),
                               win_vals, win_mass, False)
    if not traversal_opt:
        return L
    if 2 * S >= nnz or gap_lb == M:
        return L
    if gap_L == M:
        return max(0, L - M)
    Y = min(L + gap_L, INF)
    best, max_p = L, 0.0
    vals = [int(v) for v in win_vals]
    mass = [int(m) for m in win_mass]
    # sumD(x) = S + degree mass settled in [x, L): suffix sums over the window
    suffix = [0] * (len(vals) + 1)
    for i in range(len(vals) - 1, -1, -1):
        suffix[i] = suffix[i + 1] + mass[i]
    for i, x in enumerate(vals):
        p = profit(x, L, Y, S, S + suffix[i], M, nnz)
        if p > max_p:
            best, max_p = x, p
    return best


# ------------------------------------------ the selection-threshold grid --

def f32(bits: int) -> float:
    """The value of a binary32 bit pattern, as a Python (double) float."""
    return float(np.asarray(bits, dtype=np.uint32).view(np.float32))


def _value(key: int, is_f32: bool) -> float:
    return f32(key) if is_f32 else float(key)


def _values(keys: np.ndarray, is_f32: bool) -> np.ndarray:
    k = np.asarray(keys)
    if is_f32:
        return k.astype(np.uint32).view(np.float32).astype(np.float64)
    return k.astype(np.float64)


def grid_bin(key: int, inv: float, is_f32: bool = True):
    """bin(d) = floor(value(d) * inv) for inv = ST_NUM / maxW, in double; None
    past 2^31 bins, for +inf and for the sentinel.  value() is the binary32
    value of a bit pattern, or the integer itself."""
    if key >= (F32_INF_BITS if is_f32 else INF):
        return None
    x = _value(key, is_f32) * inv
    return int(math.floor(x)) if x < 2147483648.0 else None


def profit_f(x: float, L: float, Y: float, S: int, Sx: int, M: float, nnz: int) -> float:
    """Eq. (4)-(6) with real-valued ends, for a grid point x at or above about
    L - M (there lb_0 = max(x, L - M) changes no term)."""
    ub0 = min(Y, L + M)
    ub1 = min(Y, x + M)
    pushed = (ub0 - L) * float(Sx - S) / M
    pulled = (ub1 - x) * float(S) / M
    long_ = pulled * float(Sx - S) / float(nnz)
    return (pushed - long_) - pulled


def compute_st_grid(L: int, gap_L: int, gap_lb: int, S: int, nnz: int, M: int, lb0: int, Y: int,
                    settled_keys: np.ndarray, settled_deg: np.ndarray, is_f32: bool,
                    traversal_opt: bool = True) -> int:
    """Function 2 (computeST) over the ST_NUM grid (Section 4.1).  Keys are
    binary32 bit patterns (is_f32) or integers; settled_keys / settled_deg:
    settled vertices (dist < L), any of them, or one entry per distinct
    distance with its total degree."""
    inf_key = F32_INF_BITS if is_f32 else INF
    if not traversal_opt or M == 0 or L >= inf_key:
        return L
    if 2 * S >= nnz or gap_lb == M:
        return L
    if gap_L == M:
        return lb0
    inv = float(ST_NUM) / _value(M, is_f32)
    kL = grid_bin(L, inv, is_f32)
    if kL is None:
        return L
    klo = 0 if lb0 == 0 else grid_bin(lb0 - 1, inv, is_f32) + 1   # first bin with no key below lb0
    if klo > kL:
        return L
    b = np.floor(_values(settled_keys, is_f32) * inv).astype(np.int64)
    sel = (b >= klo) & (b <= kL)
    mass = {}
    for k, m in zip(b[sel].tolist(), np.asarray(settled_deg, dtype=np.int64)[sel].tolist()):
        mass[k] = mass.get(k, 0) + m
    Mf, Lf = _value(M, is_f32), _value(L, is_f32)
    Yf = math.inf if Y >= inf_key else _value(Y, is_f32)
    delta = Mf / float(ST_NUM)
    keys = sorted(mass)
    suffix, acc = {}, 0
    for k in reversed(keys):
        acc += mass[k]
        suffix[k] = acc
    best, max_p = None, 0.0
    for k in keys:
        p = profit_f(float(k) * delta, Lf, Yf, S, S + suffix[k], Mf, nnz)
        if p > max_p:
            best, max_p = k, p
    if best is None:
        return L
    lo, hi = 0, L   # smallest key whose bin is at least best
    while lo < hi:
        mid = (lo + hi) // 2
        if grid_bin(mid, inv, is_f32) >= best:
            hi = mid
        else:
            lo = mid + 1
    return lo


def compute_st_f32(L: int, gap_L: int, gap_lb: int, S: int, nnz: int, M: int, lb0: int, Y: int,
                   settled_dist: np.ndarray, settled_deg: np.ndarray,
                   traversal_opt: bool = True) -> int:
    """Function 2 (computeST) with binary32 distances (bit patterns), over the
    ST_NUM grid.  settled_dist / settled_deg: the settled vertices (dist < L)."""
    return compute_st_grid(L, gap_L, gap_lb, S, nnz, M, lb0, Y, settled_dist, settled_deg, True,
                           traversal_opt)
