"""GPU parity: distances bit-exact with the Dijkstra oracle, the schedule equal
to the sequential model's, and the preprocessing equal to its definition.
Everything is called through the C ABI (via the ctypes binding)."""
import numpy as np
import pytest

import graphgen
from graphgen import small
from oracle import eic, native
from oracle import heuristic as H

from _fixtures import INF, all_fixtures

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402


def oracle_dist(el, s):
    return native.dijkstra(el.n, el.src, el.dst, el.w, int(s))


def gpu_dist(g, s, **opts):
    return g.solve(int(s), **opts).cpu().numpy()


def assert_same(got, ref, what):
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError("%s: %d of %d differ; first %s: got %s want %s"
                             % (what, bad.shape[0], got.shape[0], bad[:5], got[bad[:5]], ref[bad[:5]]))


@pytest.mark.parametrize("fx", all_fixtures(), ids=lambda f: f["name"])
def test_golden_fixtures(fx):
    el = graphgen.from_arrays(fx["n"], fx["src"], fx["dst"], fx["w"])
    csr = graphgen.to_csr(el)
    g = sssp.Graph.from_csr(csr)
    dist = g.solve(fx["s"])
    if fx["overflow"]:
        with pytest.raises(sssp.SSSPError) as ei:
            sssp.counters()
        assert ei.value.status == -4
        return
    sssp.counters()
    assert_same(dist.cpu().numpy(), fx["dist"], fx["name"])


def test_tiny_fuzz_every_source():
    cases = 0
    for n in range(1, 11):
        for m in (0, n, 3 * n):
            for weights in ([1], [1, 2, 3], list(range(1, 256)), [0, 1, 2]):
                el = small.tiny_random(n, m, weights, seed=131 * n + m + len(weights))
                g = sssp.Graph.from_csr(graphgen.to_csr(el))
                for s in range(n):
                    assert_same(gpu_dist(g, s), oracle_dist(el, s), "n=%d m=%d s=%d" % (n, m, s))
                    cases += 1
                g.close()
    assert cases > 500


@pytest.mark.parametrize("topt", [True, False])
def test_rmat14_bit_exact(topt):
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    for s in wl.sources(8):
        assert_same(gpu_dist(g, s, traversal_opt=topt), oracle_dist(wl.edges, s), "rmat14 s=%d" % s)
        c = sssp.counters()
        assert c["flags"] == 0


def test_rmat14_host_driven_mode():
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    for s in wl.sources(2):
        assert_same(gpu_dist(g, s, host_driven=True), oracle_dist(wl.edges, s), "host-driven")


@pytest.mark.parametrize("name", ["rmat14", "er12", "grid64", "rmat12", "rmat12p1", "rmat12p4",
                                  "rmat12p17", "rmat14p20", "grid64w1000000"])
def test_schedule_matches_model(name):
    """The per-step <lb, ub, st> and the statistics taken at each step's end
    are determined by the settled set, so the GPU must reproduce the
    sequential model step for step."""
    wl = graphgen.workload(name)
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    for s in wl.sources(3):
        ref = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s))
        g.solve(int(s))
        got = sssp.schedule()
        assert len(got) == len(ref.steps), (len(got), len(ref.steps))
        for a, b in zip(got, ref.steps):
            assert (a["lb"], a["ub"], a["st"]) == (b.lb, b.ub, b.st), (a, b)
            if b.ub != INF or b.lb != 0:
                assert (a["L"], a["S"], a["h"], a["gap"], a["st_next"]) == \
                    (b.L, b.S, b.h, b.gap, b.st_next), (a, b)


def test_prep_matches_definitions():
    wl = graphgen.workload("rmat12")
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    info = g.info()
    deg = c.degrees()
    assert info["n"] == c.n and info["nnz"] == c.nnz
    assert info["max_weight"] == int(c.w.max())
    assert info["high_d0"] == H.high_d(deg)
    assert info["nonisolated"] == int((deg > 0).sum())
    assert np.array_equal(g.rtow(), H.rtow_table(c.w))
    col, w = g.sorted_rows()
    rows = np.repeat(np.arange(c.n), deg)
    order = np.lexsort((c.col, c.w, rows))
    assert np.array_equal(col, c.col[order]) and np.array_equal(w, c.w[order])
    # the internal hub-first order: rows of at least 4x the mean degree (and
    # 64) in front, at most 2^19; the rows above came back in the caller's ids
    thr = max(64, 4 * c.nnz // c.n)
    assert info["hub_first"] == min(int((deg >= thr).sum()), 1 << 19) > 0


@pytest.mark.parametrize("name", ["er16", "grid256", "rmat16"])
def test_hub_first_order_only_on_skewed_graphs(name):
    wl = graphgen.workload(name)
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    deg = c.degrees()
    thr = max(64, 4 * c.nnz // c.n)
    assert g.info()["hub_first"] == min(int((deg >= thr).sum()), 1 << 19)
    assert (g.info()["hub_first"] > 0) == name.startswith("rmat")


def test_prep_long_rows_sorted():
    """Rows longer than one LDS tile take the merge path."""
    rng = np.random.default_rng(8)
    n = 30000
    hubs = rng.integers(0, n, size=3)
    src = np.concatenate([np.repeat(hubs, 9000), rng.integers(0, n, size=20000)])
    dst = np.concatenate([rng.integers(0, n, size=27000), rng.integers(0, n, size=20000)])
    w = rng.integers(0, 2 ** 32 - 1, size=src.shape[0], dtype=np.uint64)
    el = graphgen.from_arrays(n, src, dst, w)
    c = graphgen.to_csr(el)
    g = sssp.Graph.from_csr(c)
    col, ww = g.sorted_rows()
    rows = np.repeat(np.arange(c.n), c.degrees())
    order = np.lexsort((c.col, c.w, rows))
    assert np.array_equal(col, c.col[order]) and np.array_equal(ww, c.w[order])
    assert np.array_equal(g.rtow(), H.rtow_table(c.w))


@pytest.mark.parametrize("name", ["er16", "grid256", "rmat16", "grid256w1000000"])
def test_medium_graphs_bit_exact(name):
    wl = graphgen.workload(name)
    g = sssp.Graph.from_csr(wl.csr)
    for s in wl.sources(3):
        assert_same(gpu_dist(g, s), oracle_dist(wl.edges, s), "%s s=%d" % (name, s))
        assert sssp.counters()["flags"] == 0


@pytest.mark.parametrize("power", [1, 2, 3, 4, 6, 8, 10, 17, 20])
def test_integer_power_variants_bit_exact(power):
    """The paper's integer-power variant graphs (Eq. 7; power 1 is unit weights,
    every shortest path tied), with and without the traversal filter; powers
    17 and 20 put the largest weight beyond the exact selection-threshold
    window (the ST_NUM grid)."""
    wl = graphgen.workload("rmat14p%d" % power)
    g = sssp.Graph.from_csr(wl.csr)
    for s in wl.sources(3):
        ref = oracle_dist(wl.edges, s)
        for topt in (True, False):
            assert_same(gpu_dist(g, s, traversal_opt=topt), ref, "rmat14p%d s=%d" % (power, s))
            assert sssp.counters()["flags"] == 0


def test_edge_cases():
    wl = graphgen.workload("rmat13")
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    deg = c.degrees()
    hub = int(np.argmax(deg))
    assert_same(gpu_dist(g, hub), oracle_dist(wl.edges, hub), "hub source")
    iso = int(np.nonzero(deg == 0)[0][0])
    d = gpu_dist(g, iso)
    assert d[iso] == 0 and np.all(np.delete(d, iso) == INF)
    leaf = int(np.nonzero(deg == 1)[0][0])
    assert_same(gpu_dist(g, leaf), oracle_dist(wl.edges, leaf), "leaf source")
    # zero weights, parallel edges, self-loops and several components
    el = small.disjoint_union(small.tiny_random(300, 1500, [0, 0, 1, 5, 9], seed=3),
                              small.lattice(20, 20, 3))
    g2 = sssp.Graph.from_csr(graphgen.to_csr(el))
    for s in (0, 17, 299, 300, 555):
        assert_same(gpu_dist(g2, s), oracle_dist(el, s), "zero/multi s=%d" % s)
    # weights near the top of the range, distances still representable
    el3 = small.path(4, [2 ** 30, 2 ** 30, 2 ** 31 - 2])
    g3 = sssp.Graph.from_csr(graphgen.to_csr(el3))
    assert_same(gpu_dist(g3, 0), oracle_dist(el3, 0), "large weights")


def test_batch_equals_single():
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    srcs = wl.sources(16)
    out = g.solve_batch(srcs).cpu().numpy()
    for i, s in enumerate(srcs):
        assert_same(out[i], oracle_dist(wl.edges, s), "batch row %d" % i)
    assert sssp.counters()["flags"] == 0


def test_multi_graph_batch():
    wls = [graphgen.workload("rmat%d" % s) for s in (10, 11, 12, 13)] + [graphgen.workload("grid40")]
    gs = [sssp.Graph.from_csr(w.csr) for w in wls]
    srcs = [int(w.sources(1)[0]) for w in wls]
    outs = sssp.solve_multi(gs, srcs)
    for w, s, o in zip(wls, srcs, outs):
        assert_same(o.cpu().numpy(), oracle_dist(w.edges, s), w.name)


def test_errors_are_reported_before_work():
    wl = graphgen.workload("rmat10")
    c = wl.csr
    with pytest.raises(sssp.SSSPError) as ei:
        bad = c.rowptr.copy()
        bad[5], bad[6] = bad[6], bad[5] + 100
        sssp.Graph(bad, c.col, c.w)
    assert ei.value.status in (-1,)
    with pytest.raises(sssp.SSSPError) as ei:
        w2 = c.w.copy()
        w2[0] += 1  # breaks the (u, v, w) / (v, u, w) pairing
        sssp.Graph(c.rowptr, c.col, w2)
    assert ei.value.status == -2
    g = sssp.Graph.from_csr(c)
    with pytest.raises(sssp.SSSPError) as ei:
        g.solve(c.n)
    assert ei.value.status == -1
    with pytest.raises(sssp.SSSPError):
        g.solve(-1)


def test_repeated_solves_identical():
    """Relaxation order varies run to run; the distances may not."""
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    s = int(wl.sources(1)[0])
    first = gpu_dist(g, s)
    for _ in range(5):
        assert np.array_equal(gpu_dist(g, s), first)


@pytest.mark.parametrize("name", ["grid256", "rmat14", "er12"])
def test_fused_rounds_on_off(name):
    """Bucket fusion only regroups rounds: same distances, same schedule."""
    wl = graphgen.workload(name)
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    for s in wl.sources(2):
        ref = oracle_dist(wl.edges, s)
        on = gpu_dist(g, s)
        c_on = sssp.counters()
        sched_on = sssp.schedule()
        off = gpu_dist(g, s, fuse_rounds=-1)
        c_off = sssp.counters()
        sched_off = sssp.schedule()
        assert_same(on, ref, "%s fused s=%d" % (name, s))
        assert_same(off, ref, "%s unfused s=%d" % (name, s))
        assert c_off["fused_rounds"] == 0
        assert [(a["lb"], a["ub"], a["st"]) for a in sched_on] == \
            [(a["lb"], a["ub"], a["st"]) for a in sched_off]
        if name == "grid256":
            assert c_on["fused_rounds"] > 0 and c_on["ticks"] < c_off["ticks"]


@pytest.mark.parametrize("name", ["rmat14", "grid256", "er14", "rmat14f"])
def test_tile_shapes_agree(name):
    """Every tile shape (engine instantiation: round batches of 256, 512 or
    1024 items, settle batches of 1024 or 2048) gives the oracle's distances
    and the same schedule; trees and point-to-point queries too."""
    wl = graphgen.workload(name)
    c = wl.csr
    fw = graphgen.binary32_weights(name)
    g = sssp.Graph.from_csr(c, float_weights=fw)
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    for s in wl.sources(2):
        s = int(s)
        ref = adj.dijkstra_f32(s) if fw else adj.dijkstra(s)
        scheds = []
        for shape in (1, 2, 3, 4):
            d = g.solve(s, tile_shape=shape).cpu().numpy()
            assert sssp.counters()["flags"] == 0
            assert_same(d, ref, "%s shape %d s=%d" % (name, shape, s))
            scheds.append([(a["lb"], a["ub"], a["st"]) for a in sssp.schedule()])
            dt, p = g.solve_tree(s, tile_shape=shape)
            assert_same(dt.cpu().numpy(), ref, "%s tree shape %d" % (name, shape))
            if not fw:
                assert native.check_tree(c.n, c.rowptr, c.col, c.w, s, ref, p.cpu().numpy()) == [0, 0, 0, 0]
        assert all(x == scheds[0] for x in scheds)
    # several instances of one launch, each shape
    srcs = [int(x) for x in wl.sources(3)]
    for shape in (2, 3):
        outs = sssp.solve_multi([g] * 3, srcs, tile_shape=shape)
        for s, o in zip(srcs, outs):
            ref = adj.dijkstra_f32(s) if fw else adj.dijkstra(s)
            assert_same(o.cpu().numpy(), ref, "%s multi shape %d" % (name, shape))
    adj.close()
    with pytest.raises(sssp.SSSPError):
        g.solve(srcs[0], tile_shape=9)


def test_grid_beyond_the_window_tiny_fuzz():
    """Integer weights above 65536 (the ST_NUM grid): every source of tiny
    random graphs, distances against the oracle and the schedule against the
    model."""
    cases = 0
    for n in range(2, 10):
        for m in (n, 3 * n):
            for weights in ([70000, 1, 300000], [65537, 65538, 2], [1 << 20, 70000, 1 << 19]):
                el = small.tiny_random(n, m, weights, seed=613 * n + m + weights[0] % 97)
                c = graphgen.to_csr(el)
                g = sssp.Graph.from_csr(c)
                for s in range(n):
                    assert_same(gpu_dist(g, s), oracle_dist(el, s), "n=%d m=%d s=%d" % (n, m, s))
                    ref = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, s)
                    steps = [b for b in ref.steps if not (b.lb == 0 and b.ub == INF)]
                    got = sssp.schedule()
                    # the engine keeps the first 2^16 steps (weights {1, 70000, ...}
                    # give gap-1 steps up to 70000)
                    assert len(got) == min(len(steps), 1 << 16)
                    for a, b in zip(got, steps):
                        assert (a["lb"], a["ub"], a["st"]) == (b.lb, b.ub, b.st), (n, m, s, a, b)
                    cases += 1
                g.close()
    assert cases > 150


@pytest.mark.parametrize("mode", [None, True, False])
@pytest.mark.parametrize("name", ["rmat14", "rmat12p16", "er12", "grid64w10000"])
def test_schedule_matches_model_for_each_st_candidate_set(name, mode):
    """computeST's candidates for integer weights (sssp_options.st_grid): by
    the weights (the exact window up to maxW 1024, the ST_NUM grid above), the
    grid, or the window; the engine's schedule equals the model's in the same
    mode, and the distances stay exact."""
    wl = graphgen.workload(name)
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    for s in wl.sources(3):
        ref = eic.eic_sssp(c.n, c.rowptr, c.col, c.w, int(s), st_grid=mode)
        d = g.solve(int(s), st_grid=mode)
        assert np.array_equal(d.cpu().numpy(), ref.dist)
        got = sssp.schedule()
        assert len(got) == len(ref.steps), (len(got), len(ref.steps))
        for a, b in zip(got, ref.steps):
            assert (a["lb"], a["ub"], a["st"]) == (b.lb, b.ub, b.st), (a, b)
            if b.ub != INF or b.lb != 0:
                assert (a["L"], a["S"], a["h"], a["gap"], a["st_next"]) == \
                    (b.L, b.S, b.h, b.gap, b.st_next), (a, b)
