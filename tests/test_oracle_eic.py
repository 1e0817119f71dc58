"""Pins for the sequential model of the heuristic algorithm (Section 3.3):
exact distances, the paper's behaviour bands (Section 4.3-4.5), and the
schedule's structural properties."""
import math

import numpy as np
import pytest

import graphgen
from graphgen import small
from oracle import eic, native
from oracle import heuristic as H

INF = H.INF


def _csr_run(el, s, **kw):
    c = graphgen.to_csr(el)
    return c, eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, **kw)


@pytest.mark.parametrize("topt", [True, False])
def test_model_exact_on_tiny_fuzz(topt):
    for n in range(1, 11):
        for m in (0, n, 3 * n):
            for weights in ([1], [1, 2, 3], list(range(1, 256)), [0, 1, 2]):
                el = small.tiny_random(n, m, weights, seed=97 * n + m + len(weights))
                c = graphgen.to_csr(el)
                for s in range(n):
                    ref = native.dijkstra(el.n, el.src, el.dst, el.w, s)
                    got = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, traversal_opt=topt).dist
                    assert np.array_equal(got, ref), (n, m, weights[:3], s)


@pytest.mark.parametrize("name", ["rmat14", "er13", "grid96", "rmat12"])
@pytest.mark.parametrize("topt", [True, False])
def test_model_exact_on_workloads(name, topt):
    wl = graphgen.workload(name)
    c = wl.csr
    for s in wl.sources(3):
        ref = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, int(s))
        got = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s), traversal_opt=topt).dist
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("beta", [0.85, 0.95])
@pytest.mark.parametrize("alpha", [1, 3, 8])
def test_model_exact_for_other_constants(alpha, beta):
    wl = graphgen.workload("rmat12")
    c = wl.csr
    s = int(wl.sources(1)[0])
    ref = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, s)
    got = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, alpha=alpha, beta=beta).dist
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", ["rmat14", "er14", "rmat16"])
def test_model_within_the_papers_bands(name):
    """Section 4.3: nFrontier 1.01-1.10 on the low-diameter benchmark graphs
    (worst 1.20 over all variants) and nSync 1.55-6.13 (0.54-3.64 on the
    variants); Section 4.4: nTrav about 3-5.4 and below |E|/|V|/2 whenever
    there are enough skippable edges."""
    wl = graphgen.workload(name)
    c = wl.csr
    deg = c.degrees()
    half_ev = (c.nnz / 2) / int((deg > 0).sum()) / 2
    for s in wl.sources(3):
        r = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s))
        k = eic.normalised(r, c.n, deg)
        assert 1.0 <= k["nFrontier"] < 1.20, k
        assert 0.5 <= k["nSync"] <= 6.2, k
        assert 2.5 <= k["nTrav"] <= 5.5, k
        assert k["nTrav"] < half_ev, (k, half_ev)


def test_traversal_optimisation_cuts_traversals():
    """Section 4.4: with the selection threshold the traversals per reachable
    vertex fall well below the push-only count on a skewed graph."""
    wl = graphgen.workload("rmat14")
    c = wl.csr
    s = int(wl.sources(1)[0])
    on = eic.normalised(eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s), c.n, c.degrees())
    off = eic.normalised(eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, traversal_opt=False),
                         c.n, c.degrees())
    assert on["nTrav"] < 0.5 * off["nTrav"]


def test_schedule_structure():
    """lb grows by the gap, st <= lb, the band width is gap(lb), and the loop
    stops at the first step end with max finite dist + M < lb."""
    wl = graphgen.workload("er13")
    c = wl.csr
    M = int(c.w.max())
    for s in wl.sources(2):
        r = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s))
        steps = r.steps
        assert steps[0].lb == 0 and steps[0].st == 0
        for a, b in zip(steps, steps[1:]):
            assert b.lb == a.L
            assert b.ub == min(a.L + a.gap, INF)
            assert b.st == a.st_next
            assert 0 <= b.st <= b.lb
            assert 1 <= a.gap <= M
        for a in steps[1:]:
            assert a.L > a.lb
        maxfin = int(r.dist[r.dist != INF].max())
        assert maxfin + M < steps[-1].L + steps[-1].gap
        # the step before the last had not yet met the stopping rule
        if len(steps) >= 2:
            assert not (maxfin + M < steps[-2].L)


def test_hub_source_terminates():
    """A source of degree >= highD(0) makes the first step's ub collapse to 0
    (the hub update reads dist[s] = 0); the loop must still advance."""
    wl = graphgen.workload("rmat12")
    c = wl.csr
    deg = c.degrees()
    hub = int(np.argmax(deg))
    ref = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, hub)
    r = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, hub, max_steps=10_000)
    assert np.array_equal(r.dist, ref)
    assert r.steps[0].L == 0
    assert len(r.steps) < 1000


def test_no_hub_reachable_ends_after_first_step():
    """A component with only low-degree vertices never meets a vertex of
    degree >= highD(0): the first step relaxes everything with ub = +inf."""
    big = graphgen.workload("rmat10").edges
    el = small.disjoint_union(big, small.path(20, np.arange(1, 20)))
    c = graphgen.to_csr(el)
    s = big.n  # start of the path
    r = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s)
    ref = native.dijkstra(el.n, el.src, el.dst, el.w, s)
    assert np.array_equal(r.dist, ref)
    assert len(r.steps) == 1 and r.steps[0].ub == INF


def test_model_on_integer_power_variants():
    """Section 4.4 on the integer-power variant graphs (Eq. 7): traversals per
    reachable vertex are worst with a single weight (power 1: every shortest
    path ties, each edge is scanned from both sides) and about 3-5.5 once there
    are at least 255 distinct weights; distances stay exact throughout."""
    ntrav = {}
    for p in (1, 4, 8, 10):
        wl = graphgen.workload("rmat14p%d" % p)
        c = wl.csr
        vals = []
        for s in wl.sources(2):
            r = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s))
            ref = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, int(s))
            assert np.array_equal(r.dist, ref), (p, s)
            vals.append(eic.normalised(r, c.n, c.degrees())["nTrav"])
        ntrav[p] = float(np.mean(vals))
    assert ntrav[1] > 4 * ntrav[10], ntrav
    assert ntrav[1] > ntrav[4] > ntrav[8] * 0.9, ntrav
    for p in (8, 10):
        assert 2.5 <= ntrav[p] <= 5.5, ntrav


@pytest.mark.parametrize("name", ["rmat12p17", "rmat12p20"])
def test_weights_beyond_the_exact_window_use_the_grid(name):
    """Weights above 65536 (Eq. 7 with power 17 and 20): computeST runs on the
    ST_NUM grid, the model pulls and scans far fewer entries than with the
    traversal optimisation off, and stays exact."""
    wl = graphgen.workload(name)
    c = wl.csr
    assert int(c.w.max()) > 65536
    deg = c.degrees()
    for s in wl.sources(2):
        ref = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, int(s))
        on = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s))
        off = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s), traversal_opt=False)
        assert np.array_equal(on.dist, ref) and np.array_equal(off.dist, ref)
        assert on.pulls > 0
        assert eic.normalised(on, c.n, deg)["nTrav"] < 0.5 * eic.normalised(off, c.n, deg)["nTrav"]


def test_st_grid_model_is_exact():
    """computeST on the ST_NUM grid for integer weights within the exact
    window's range (st_grid): another schedule, the same distances."""
    for n in range(2, 11):
        for weights in ([1, 2, 3], list(range(1, 256)), [0, 1, 2]):
            el = small.tiny_random(n, 3 * n, weights, seed=31 * n + len(weights))
            c = graphgen.to_csr(el)
            for s in range(n):
                ref = native.dijkstra(el.n, el.src, el.dst, el.w, s)
                got = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, st_grid=True).dist
                assert np.array_equal(got, ref), (n, weights[:3], s)
    wl = graphgen.workload("rmat12p16")
    c = wl.csr
    assert 1024 < int(c.w.max()) <= 65536
    for s in wl.sources(2):
        ref = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, int(s))
        assert np.array_equal(eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s), st_grid=True).dist, ref)


def test_st_grid_equals_the_window_when_bins_are_no_wider_than_one():
    """With ST_NUM = 1024 bins per maxW and maxW <= 1024 a bin is at most one
    distance unit wide, so each bin holds at most one integer distance: the
    grid's candidates and their masses are the exact window's, scored at the
    grid point at or just below each distance (at the distance itself when
    maxW = 1024), and every step here picks the same threshold. Wider bins
    (maxW up to 65536) give another schedule."""
    rng = np.random.default_rng(3)
    for t in range(40):
        n = int(rng.integers(5, 160))
        m = int(rng.integers(n, 5 * n))
        top = int(rng.choice([255, 1000, 1024]))
        el = small.tiny_random(n, m, list(range(1, top + 1)), seed=1000 + t)
        c = graphgen.to_csr(el)
        s = int(rng.integers(0, n))
        a = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s)
        b = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, st_grid=True)
        assert [(x.lb, x.ub, x.st, x.st_next) for x in a.steps] == \
               [(x.lb, x.ub, x.st, x.st_next) for x in b.steps], (t, top)
    wl = graphgen.workload("rmat12p16")
    c = wl.csr
    s = int(wl.sources(1)[0])
    a = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, st_grid=False)
    b = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s, st_grid=True)
    assert [x.st_next for x in a.steps] != [x.st_next for x in b.steps]
    # above ST_NUM the grid is the default
    d = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s)
    assert [x.st_next for x in d.steps] == [x.st_next for x in b.steps]
