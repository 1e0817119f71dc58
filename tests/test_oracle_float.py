"""Pins for the oracle's binary32 Dijkstra (real weights: the gr26 graphs'
(0, 1] weights and the float-pivot variants of Eq. 8): Bellman-Ford in
binary32 on exhaustive tiny fuzz, exact sums of dyadic weights, integer-valued
weights against the integer Dijkstra, the in-order rounding of a path sum, and
the weight generators (Eq. 8's bell curve around the pivot)."""
import numpy as np
import pytest

import graphgen
from graphgen import small
from oracle import native

INF = 0xFFFFFFFF


def bellman_ford_f32(n, src, dst, wbits, s):
    """|V|-1 rounds of relaxing every edge both ways, each sum one binary32
    addition (numpy float32 scalars)."""
    w = wbits.view(np.float32)
    d = [None] * n
    d[s] = np.float32(0.0)
    for _ in range(max(n - 1, 1)):
        changed = False
        for u, v, c in zip(src.tolist(), dst.tolist(), w.tolist()):
            c = np.float32(c)
            for a, b in ((u, v), (v, u)):
                if d[a] is not None:
                    t = np.float32(d[a] + c)
                    if d[b] is None or t < d[b]:
                        d[b] = t
                        changed = True
        if not changed:
            break
    out = np.full(n, INF, np.uint32)
    for v in range(n):
        if d[v] is not None:
            out[v] = np.array([d[v]], np.float32).view(np.uint32)[0]
    return out


VALUE_SETS = {
    "dyadic": [0.5, 0.25, 0.125, 1.0],
    "decimal": [0.1, 0.2, 0.7, 1e-3],
    "with_zero": [0.0, 0.3, 0.33333334],
    "wide": [16777216.0, 1.0, 3.0, 0.5],
}


@pytest.mark.parametrize("vname", sorted(VALUE_SETS))
def test_f32_dijkstra_matches_f32_bellman_ford(vname):
    vals = np.asarray(VALUE_SETS[vname], np.float32)
    for n in range(1, 10):
        for m in (0, n, 3 * n):
            el = small.tiny_random(n, m, [1], seed=4000 + 10 * n + m)
            rng = np.random.default_rng(4100 + 10 * n + m)
            wb = rng.choice(vals, size=el.src.shape[0]).view(np.uint32)
            adj = native.Adjacency(n, el.src, el.dst, wb)
            for s in range(n):
                assert np.array_equal(adj.dijkstra_f32(s), bellman_ford_f32(n, el.src, el.dst, wb, s)), (vname, n, m, s)
            adj.close()


def test_dyadic_path_sums_are_exact():
    el = small.path(6, [1, 1, 1, 1, 1])
    wb = np.array([0.5, 0.25, 0.125, 0.0625, 2.0], np.float32).view(np.uint32)
    adj = native.Adjacency(6, el.src, el.dst, wb)
    assert adj.dijkstra_f32(0).view(np.float32).tolist() == [0.0, 0.5, 0.75, 0.875, 0.9375, 2.9375]


def test_integer_valued_weights_agree_with_the_integer_dijkstra():
    for seed in range(5):
        el = small.tiny_random(40, 120, list(range(0, 200)), seed=900 + seed)
        wb = el.w.astype(np.float32).view(np.uint32)
        adj = native.Adjacency(40, el.src, el.dst, wb)
        for s in (0, 7, 31):
            ref = native.dijkstra(40, el.src, el.dst, el.w, s)
            got = adj.dijkstra_f32(s)
            fin = ref != INF
            assert np.array_equal(got == INF, ~fin)
            assert np.array_equal(got[fin].view(np.float32), ref[fin].astype(np.float32))
        adj.close()


def test_sums_round_in_path_order():
    # 2^24 + 1 rounds to 2^24 (ties to even) at every step, so the far end of
    # 0 -(2^24)- 1 -(1)- 2 -(1)- 3 stays at 2^24 and beats the direct 2^24 + 4
    el = graphgen.from_arrays(4, [0, 1, 2, 0], [1, 2, 3, 3],
                              np.array([16777216.0, 1.0, 1.0, 16777220.0], np.float32).view(np.uint32))
    adj = native.Adjacency(4, el.src, el.dst, el.w)
    assert adj.dijkstra_f32(0).view(np.float32).tolist() == [0.0, 16777216.0, 16777216.0, 16777216.0]


@pytest.mark.parametrize("pivot", [None, 0.1, 0.5, 0.9])
def test_real_weight_generators(pivot):
    """Uniform on (0, 1]; Eq. 8 maps it to a bell curve peaking at the pivot
    with half of the weights below it; repeatable; valid binary32 values."""
    m = 300000
    wb = graphgen.weights_f32(m, 77, pivot)
    assert np.array_equal(wb, graphgen.weights_f32(m, 77, pivot))
    w = wb.view(np.float32)
    assert np.all(np.isfinite(w)) and w.min() > 0.0 and w.max() <= 1.0
    med = float(np.median(w))
    if pivot is None:
        assert abs(med - 0.5) < 0.01
        assert abs(float(np.mean(w)) - 0.5) < 0.01
    else:
        assert abs(med - pivot) < 0.01
        # the density peaks at the pivot: more weights within 0.05 of it than
        # in any other window of that width
        hist, _ = np.histogram(w, bins=20, range=(0.0, 1.0))
        assert abs((np.argmax(hist) + 0.5) / 20 - pivot) <= 0.05 + 1e-9, hist
