"""Pins for the oracle's statistics and heuristics (Sections 3.1, 3.2, 3.3, 4.1)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import graphgen
from oracle import heuristic as H


# ---------------------------------------------------------------- highD ----

def highd_brute(degs):
    """Every integer threshold h: low = {deg < h}, high = {deg >= h}; keep the
    thresholds that are degrees present in the set; least |low - high| mass,
    smallest such h."""
    degs = [int(d) for d in degs if d >= 1]
    if not degs:
        return 0
    best = None
    for h in sorted(set(degs)):
        low = sum(d for d in degs if d < h)
        high = sum(d for d in degs if d >= h)
        key = (abs(low - high), h)
        if best is None or key < best:
            best = key
    return best[1]


def test_highd_matches_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(300):
        k = int(rng.integers(0, 40))
        degs = rng.integers(0, int(rng.integers(1, 30)) + 1, size=k)
        assert H.high_d(degs) == highd_brute(degs), degs


def test_highd_regular_graph_is_its_degree():
    for d in (1, 2, 3, 7, 32):
        assert H.high_d(np.full(1000, d)) == d


def test_highd_uniform_random_graph_matches_table1_urand():
    """Table 1: Urand (uniform random, mean degree 32) has highD(0) = 33."""
    el = graphgen.gnm(1 << 16, 16 << 16, seed=7)
    csr = graphgen.to_csr(el)
    assert H.high_d(csr.degrees()) == 33


def test_highd_rmat_scale26_matches_table1_gr26_4():
    """Table 1, gr26_4 (Graph500 Kronecker, scale 26, edge factor 4):
    |V| = 21.7 M non-isolated, max degree 426944, highD(0) = 417. The same
    recipe (a, b, c) = (0.57, 0.19, 0.19) through our generator, degrees of the
    multigraph (parallel edges counted, self-loops dropped)."""
    deg = graphgen.rmat_degrees(26, 4, seed=1)
    assert abs(int((deg > 0).sum()) - 21.7e6) < 0.05e6
    assert abs(int(deg.max()) - 426944) < 0.01 * 426944
    assert H.high_d(deg) == 417


def test_highd_empty_set_is_zero():
    assert H.high_d(np.zeros(0)) == 0
    assert H.high_d(np.zeros(10)) == 0


# --------------------------------------------------------- maxW / RtoW ----

def _count_le(ws, t):
    return int(np.count_nonzero(ws <= t))


def test_rtow_is_the_weight_quantile():
    """RtoW[x] = maxW(G, x/(RATIO_NUM-1)): at least a fraction x/4095 of the
    weights are <= RtoW[x], and fewer than that are <= RtoW[x] - 1 (for x = 0
    the threshold is the smallest weight present)."""
    rng = np.random.default_rng(5)
    for ws in (rng.integers(1, 256, size=10_000), rng.integers(0, 4, size=777),
               rng.integers(1, 2 ** 32 - 1, size=5000, dtype=np.uint64),
               np.array([9]), np.arange(1, 4097)):
        ws = np.asarray(ws, dtype=np.uint64)
        t = H.rtow_table(ws)
        nnz = ws.shape[0]
        assert t[0] == ws.min() and t[-1] == ws.max()
        for x in range(0, 4096, 37):
            need = Fraction(x * nnz, 4095)
            assert _count_le(ws, int(t[x])) >= need
            if x > 0 and t[x] > 0:
                assert _count_le(ws, int(t[x]) - 1) < need
        assert np.all(np.diff(t.astype(np.int64)) >= 0)


def test_max_w_quantile_definition():
    ws = np.arange(1, 101, dtype=np.uint64)  # 1..100
    assert H.max_w(ws, 1.0) == 100
    assert H.max_w(ws, 0.5) == 50
    assert H.max_w(ws, 0.505) == 51
    assert H.max_w(ws, 0.0) == 1


# ------------------------------------------------- Eq. (1)-(3): stepping ----

def test_prob_at_zero_is_beta():
    """sumD(0) = 2|E| (VS(0) = V), so Eq. (1) gives prob(0) = min(beta, 1)."""
    for nnz in (2, 100, 10 ** 9):
        for beta in (0.85, 0.9, 0.95):
            assert H.prob(nnz, nnz, beta) == beta


def test_prob_is_at_least_half():
    """Section 3.1: prob(lb) >= 0.5 whenever beta is in [0.5, 1)."""
    rng = np.random.default_rng(1)
    for _ in range(2000):
        nnz = int(rng.integers(1, 10 ** 12))
        S = int(rng.integers(0, nnz + 1))
        beta = float(rng.uniform(0.5, 0.999))
        assert 0.5 <= H.prob(S, nnz, beta) <= beta


def test_ratio_inverts_the_tail_bound_of_section_3_1():
    """Section 3.1 rewrites (1 - ratio)^ne as (1 - prob)^(ne / (prob * highD)):
    Eq. (2) is exactly the ratio for which that holds for every ne."""
    rng = np.random.default_rng(2)
    for _ in range(500):
        p = float(rng.uniform(0.5, 0.95))
        h = int(rng.integers(4, 10 ** 6))
        r = H.ratio(p, h)
        assert 0.0 < r < 1.0
        for ne in (1, 7, h, 3 * h):
            lhs = (1.0 - r) ** ne
            rhs = (1.0 - p) ** (ne / (p * h))
            assert math.isclose(lhs, rhs, rel_tol=1e-9, abs_tol=1e-300)


def test_gap_branches_and_range():
    ws = np.random.default_rng(4).integers(1, 256, size=50_000)
    t = H.rtow_table(ws)
    M = int(ws.max())
    nnz = ws.shape[0]
    # highD <= alpha -> maxW(G, 1) = M
    for h in (0, 1, 2, 3):
        assert H.gap(nnz, h, nnz, M, t) == M
    # highD > alpha -> the ratio-quantile of the weights, in [1, M]
    for h in (4, 8, 33, 417, 1681, 10 ** 6):
        for S in (nnz, nnz // 2, nnz // 10, 1):
            g = H.gap(S, h, nnz, M, t)
            r = H.ratio(H.prob(S, nnz), h)
            assert 1 <= g <= M
            assert g == max(1, int(t[H.ratio_index(r)]))
            assert _count_le(ws, g) >= Fraction(H.ratio_index(r) * nnz, 4095)
    # larger highD -> smaller (or equal) gap at the same sumD
    gs = [H.gap(nnz, h, nnz, M, t) for h in (4, 8, 33, 417, 1681)]
    assert gs == sorted(gs, reverse=True)


# Eq. (1)-(3) at lb = 0 (sumD(0) = 2|E|, so prob = beta = 0.9), worked by hand
# for the highD values of Table 1's graph families: ratio to six decimals, and
# gap = maxW(G, ratio) on weights spread exactly uniformly over 1..W, where the
# ratio-quantile is the smallest w with w / W >= (table index) / 4095 and the
# table index is ratio * 4095 rounded up.
WORKED_GAPS = [
    # highD, ratio,    gap on 1..255, gap on 1..1000
    (4, 0.472500, 121, 473),
    (8, 0.273708, 70, 274),
    (33, 0.074599, 20, 75),
    (417, 0.006117, 2, 7),
    (1681, 0.001521, 1, 2),
]


@pytest.mark.parametrize("copies", [1, 3])
def test_gap_worked_table(copies):
    for W, col in ((255, 2), (1000, 3)):
        ws = np.repeat(np.arange(1, W + 1, dtype=np.uint64), copies)
        nnz = int(ws.shape[0])
        t = H.rtow_table(ws)
        for row in WORKED_GAPS:
            h, r = row[0], row[1]
            got_r = H.ratio(H.prob(nnz, nnz), h)
            assert round(got_r, 6) == r, (h, got_r)
            assert H.gap(nnz, h, nnz, W, t) == row[col], (W, h, copies)


def test_gap_quantile_covers_the_ratio():
    """maxW(G, ratio) is a weight w with P(weight <= w) >= ratio (Section 3's
    definition); the 4096-entry table (Section 4.1) can only round the ratio
    up, by less than one table step. A lookup index rounded down, or a table
    built from a floor of i * nnz / 4095, breaks the first bound."""
    rng = np.random.default_rng(77)
    for trial in range(300):
        nnz = int(rng.integers(1, 3000))
        W = int(rng.choice([3, 17, 255, 1000, 70000]))
        ws = rng.integers(1, W + 1, size=nnz).astype(np.uint64)
        t = H.rtow_table(ws)
        M = int(ws.max())
        for _ in range(6):
            h = int(rng.integers(4, 5000))
            S = int(rng.integers(0, nnz + 1))
            r = H.ratio(H.prob(S, nnz), h)
            g = H.gap(S, h, nnz, M, t)
            assert Fraction(_count_le(ws, g)) >= Fraction(r) * nnz, (trial, r, g)
            # g is the smallest weight reaching the rounded-up quantile
            assert Fraction(_count_le(ws, g - 1)) < (Fraction(r) + Fraction(1, 4095)) * nnz, (trial, r, g)


def test_gap_is_at_least_one_with_zero_weights():
    ws = np.zeros(1000, dtype=np.uint64)
    t = H.rtow_table(ws)
    assert H.gap(1000, 50, 1000, 0, t) == 1
    assert H.gap(1000, 2, 1000, 0, t) == 1


# ------------------------------------ Eq. (4)-(6) and Function 2 --------

def test_compute_st_guards():
    vals = np.array([95]); mass = np.array([10])
    # sumD(L) >= |E|  (2 S >= nnz): no pull
    assert H.compute_st(100, 4, 5, 500, 1000, 10, vals, mass) == 100
    # the current gap is maxW(G, 1): no pull
    assert H.compute_st(100, 4, 10, 20, 1000, 10, vals, mass) == 100
    # the next gap is maxW(G, 1): pull from everything in [L - M, L)
    assert H.compute_st(100, 10, 5, 20, 1000, 10, vals, mass) == 90
    assert H.compute_st(4, 10, 5, 20, 1000, 10, vals, mass) == 0
    # traversal optimisation switched off
    assert H.compute_st(100, 4, 5, 20, 1000, 10, vals, mass, traversal_opt=False) == 100


def test_compute_st_hand_worked_window():
    """L = 100, M = 10, gap(L) = 4 (Y = 104), nnz = 1000, sumD(L) = S = 20.
    Settled distances in [90, 100): 92 (degree mass 300), 97 (100), 99 (50).
    Worked by hand from Eq. (4)-(6) with the Section 3.2 clamps:
      x=92: Sx-S=450, ub0=104, ub1=min(104,102)=102
            pushed=4*450/10=180  pulled=(102-92)*20/10=20  long=20*450/1000=9
            profit=151
      x=97: Sx-S=150, ub1=104: pushed=60, pulled=14, long=2.1 -> 43.9
      x=99: Sx-S=50:  pushed=20, pulled=10, long=0.5 -> 9.5
    so ST = 92."""
    vals = np.array([92, 97, 99]); mass = np.array([300, 100, 50])
    assert H.compute_st(100, 4, 5, 20, 1000, 10, vals, mass) == 92
    assert math.isclose(H.profit(92, 100, 104, 20, 470, 10, 1000), 151.0)
    assert math.isclose(H.profit(97, 100, 104, 20, 170, 10, 1000), 43.9)
    assert math.isclose(H.profit(99, 100, 104, 20, 70, 10, 1000), 9.5)


def test_compute_st_no_profit_keeps_lb():
    """A heavy unsettled side (S large against the settled window) makes the
    pulled term dominate: every profit is negative and ST stays L.
      x=95: pushed=4*10/10=4, pulled=(104-95)*400/10=360 -> negative."""
    vals = np.array([95]); mass = np.array([10])
    assert H.compute_st(100, 4, 5, 400, 1000, 10, vals, mass) == 100


def test_profit_clamps_below_the_window():
    """Below L - M every x clamps to lb_0 = L - M (Section 3.2)."""
    a = H.profit(90, 100, 104, 20, 470, 10, 1000)
    for x in (0, 50, 89):
        assert H.profit(x, 100, 104, 20, 470, 10, 1000) == a


def test_profit_nondecreasing_between_distances():
    """With sumD(x) fixed on an interval between consecutive settled
    distances, Eq. (4)-(6) never decrease as x grows: evaluating only the
    distinct distances (the candidate set of Function 2) loses nothing."""
    rng = np.random.default_rng(9)
    for _ in range(300):
        M = int(rng.integers(2, 300))
        L = int(rng.integers(M, 10 * M))
        g = int(rng.integers(1, M))
        Y = L + g
        nnz = int(rng.integers(1000, 10 ** 6))
        S = int(rng.integers(1, nnz // 2))
        Sx = S + int(rng.integers(0, nnz - S))
        xs = range(L - M, L)
        ps = [H.profit(x, L, Y, S, Sx, M, nnz) for x in xs]
        assert all(b >= a for a, b in zip(ps, ps[1:]))


# ------------------------------------------ the grid beyond the exact window

def test_integer_grid_equals_the_exact_window_on_multiples_of_the_bin_width():
    """With maxW = ST_NUM * c (beyond the exact window) and every distance,
    gap and L a multiple of c, the grid's bins are exactly the distinct
    distances, and every term of Eq. 4-6 is a ratio of exact integers, each
    scaled by c: the grid computeST returns c times the exact-window
    computeST of the problem divided by c."""
    from oracle import heuristic as Hm
    rng = np.random.default_rng(4242)
    c = 100
    Mi = Hm.ST_NUM          # the scaled-down problem (exact window)
    M = Mi * c              # 102400 > ST_WINDOW_MAX
    assert M > Hm.ST_WINDOW_MAX
    hits = 0
    for trial in range(400):
        Li = int(rng.integers(1, 6 * Mi))
        gap_i = int(rng.integers(1, Mi))
        gap_lb_i = int(rng.integers(1, Mi))
        nnz = int(rng.integers(1000, 100000))
        S = int(rng.integers(0, nnz // 2)) if trial % 2 else int(rng.integers(0, 3000))
        k = int(rng.integers(0, 200))
        settled = rng.integers(max(0, Li - Mi), Li, size=k)
        degs = rng.integers(1, 500, size=k)
        wv, inv = np.unique(settled, return_inverse=True)
        wm = np.zeros(wv.shape[0], np.int64)
        np.add.at(wm, inv, degs)
        want = Hm.compute_st(Li, gap_i, gap_lb_i, S, nnz, Mi, wv, wm)
        got = Hm.compute_st(Li * c, gap_i * c, gap_lb_i * c, S, nnz, M, wv * c, wm)
        assert got == want * c, (trial, Li, want, got)
        hits += want < Li
    assert hits > 100


def test_integer_grid_threshold_is_the_first_value_of_its_bin():
    from oracle import heuristic as Hm
    M = 3 * 65536 + 7
    inv = float(Hm.ST_NUM) / float(M)
    rng = np.random.default_rng(7)
    for _ in range(200):
        L = int(rng.integers(M // 2, 4 * M))
        settled = np.unique(rng.integers(max(0, L - M), L, size=300))
        degs = rng.integers(1, 400, size=settled.shape[0])
        st = Hm.compute_st(L, M // 50, M // 40, 2000, 10 ** 6, M, settled, degs)
        assert max(0, L - M) <= st <= L
        if st < L:
            k = Hm.grid_bin(st, inv, False)
            assert st == 0 or Hm.grid_bin(st - 1, inv, False) < k
            assert np.any((settled >= st) & (np.floor(settled * inv) == k))
