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
    "tiny": [1e-30, 3e-30, 1e-29],
    "extreme": [1e30, 1.0, 1e-30],
    "all_zero": [0.0],
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


# ------------------------------------------------ the binary32 schedule model

from oracle import eic  # noqa: E402
from oracle import heuristic as H  # noqa: E402


def _bits(x):
    return int(np.array([x], np.float32).view(np.uint32)[0])


@pytest.mark.parametrize("topt", [True, False])
def test_f32_model_reaches_the_f32_dijkstra_tiny_fuzz(topt):
    incomplete = 0
    for vname, vals in sorted(VALUE_SETS.items()):
        vals = np.asarray(vals, np.float32)
        for n in range(1, 9):
            for m in (0, n, 3 * n):
                el = small.tiny_random(n, m, [1], seed=5000 + 10 * n + m)
                rng = np.random.default_rng(5100 + 10 * n + m)
                wb = rng.choice(vals, size=el.src.shape[0]).view(np.uint32)
                el = graphgen.from_arrays(n, el.src, el.dst, wb)
                c = graphgen.to_csr(el)
                adj = native.Adjacency(n, el.src, el.dst, el.w)
                for s in range(n):
                    r = eic.eic_sssp_f32(c.n, c.rowptr, c.col, c.w, s, traversal_opt=topt,
                                         max_steps=2000)
                    if not r.complete:
                        # a band narrower than the spacing of the distances
                        # left: only weights spanning 60 decades do this
                        assert vname == "extreme", (vname, n, m, s)
                        incomplete += 1
                        continue
                    assert np.array_equal(r.dist, adj.dijkstra_f32(s)), (vname, n, m, s)
                adj.close()
    assert incomplete < 10


@pytest.mark.parametrize("name", ["rmat12f", "rmat12c1", "rmat12c5", "rmat12c9"])
def test_f32_model_workloads_pull_and_stay_exact(name):
    """With the ST_NUM grid the model pulls, scans far fewer entries than with
    the traversal optimisation off, and still reaches the binary32 Dijkstra."""
    wl = graphgen.workload(name)
    c = wl.csr
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    for s in wl.sources(2):
        ref = adj.dijkstra_f32(int(s))
        on = eic.eic_sssp_f32(c.n, c.rowptr, c.col, c.w, int(s))
        off = eic.eic_sssp_f32(c.n, c.rowptr, c.col, c.w, int(s), traversal_opt=False)
        assert np.array_equal(on.dist, ref) and np.array_equal(off.dist, ref)
        assert on.pulls > 0 and off.pulls == 0
        deg = c.degrees()
        assert eic.normalised(on, c.n, deg)["nTrav"] < 0.5 * eic.normalised(off, c.n, deg)["nTrav"]
        for st in on.steps:
            assert st.st <= st.lb
    adj.close()


def test_grid_compute_st_equals_the_exact_window_on_dyadic_distances():
    """With maxW = 1 and every distance a multiple of 1/ST_NUM, the grid's bins
    are exactly the distinct distances, and Eq. 4-6 scale by a power of two:
    the grid computeST must return the exact-window computeST of the
    distances times ST_NUM, divided by ST_NUM."""
    rng = np.random.default_rng(31337)
    Mi = H.ST_NUM
    Mb = _bits(1.0)
    hits = 0
    for trial in range(400):
        Li = int(rng.integers(1, 6 * Mi))
        gap_i = int(rng.integers(1, Mi))          # below M: the main branch
        gap_lb_i = int(rng.integers(1, Mi))
        nnz = int(rng.integers(1000, 100000))
        S = int(rng.integers(0, nnz // 2)) if trial % 2 else int(rng.integers(0, 3000))
        k = int(rng.integers(0, 200))
        settled = rng.integers(max(0, Li - Mi - 8), Li, size=k) if Li > 0 else np.zeros(0, np.int64)
        degs = rng.integers(1, 500, size=settled.shape[0])
        wv, inv = np.unique(settled[settled >= max(0, Li - Mi)], return_inverse=True)
        wm = np.zeros(wv.shape[0], np.int64)
        np.add.at(wm, inv, degs[settled >= max(0, Li - Mi)])
        want = H.compute_st(Li, gap_i, gap_lb_i, S, nnz, Mi, wv, wm)
        Lb = _bits(Li / Mi)
        Lf = np.float32(Li / Mi)
        ulp = np.float32(H.f32(Lb + 1)) - Lf
        lo = np.float32(np.float32(Lf - np.float32(1.0)) - np.float32(2.0) * ulp)
        lb0 = _bits(lo) if lo > 0 else 0
        Yb = _bits((Li + gap_i) / Mi)
        sb = np.array([_bits(x / Mi) for x in settled.tolist()], np.uint32)
        got = H.compute_st_f32(Lb, _bits(gap_i / Mi), _bits(gap_lb_i / Mi), S, nnz, Mb, lb0, Yb, sb, degs)
        assert H.f32(got) * Mi == want, (trial, Li, want, H.f32(got) * Mi)
        hits += want < Li
    assert hits > 100


def test_grid_threshold_is_the_first_value_of_its_bin():
    rng = np.random.default_rng(99)
    wl = graphgen.workload("rmat12f")
    c = wl.csr
    r = eic.eic_sssp_f32(c.n, c.rowptr, c.col, c.w, int(wl.sources(1)[0]))
    M = int(c.w.max())
    inv = float(H.ST_NUM) / H.f32(M)
    seen = 0
    for st in r.steps:
        if st.st < st.lb and st.st > 0:
            k = H.grid_bin(st.st, inv)
            assert H.grid_bin(st.st - 1, inv) < k
            seen += 1
    assert seen > 0
    # bins never decrease along the bit patterns
    x = np.sort(rng.integers(0, 0x40000000, size=20000)).tolist()
    b = [H.grid_bin(v, inv) for v in x]
    assert all(b[i] <= b[i + 1] for i in range(len(b) - 1))
