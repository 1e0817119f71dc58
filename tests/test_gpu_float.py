"""GPU solves with real weights (SSSP_CREATE_FLOAT_WEIGHTS): binary32 weights
and distances, bit-exact with the oracle's binary32 Dijkstra (each path's
weights summed in order, rounded to nearest) on tiny fuzz graphs, the gr26
stand-in (weights uniform on (0, 1]) and its float-pivot variants (Eq. 8)."""
import numpy as np
import pytest

import graphgen
from graphgen import small
from oracle import eic, native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402

INF = 0xFFFFFFFF


def f32_edges(el, values, seed):
    rng = np.random.default_rng(seed)
    w = rng.choice(np.asarray(values, dtype=np.float32), size=el.src.shape[0]).view(np.uint32)
    return graphgen.from_arrays(el.n, el.src, el.dst, w)


def assert_bits(got, ref, what):
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError("%s: %d of %d differ; first %s: got %s want %s" % (
            what, bad.shape[0], got.shape[0], bad[:4], got[bad[:4]].view(np.float32),
            ref[bad[:4]].view(np.float32)))


# The method advances its band by gap(L) per step (Section 3.3); where the
# remaining distances are spaced far wider than the weight quantiles (weights
# 1e-30 and 1e30 in one graph), the binary32 model needs a step per unit in the
# last place. Such (graph, source) cases are left out: the oracle's model
# decides, with this many steps.
MODEL_STEPS = 2000


def model_completes(c, s):
    return eic.eic_sssp_f32(c.n, c.rowptr, c.col, c.w, s, max_steps=MODEL_STEPS).complete


def test_tiny_fuzz_every_source():
    cases = skipped = 0
    sets = ([0.5, 0.25, 1.0], [0.1, 0.2, 0.7, 1e-3], [0.0, 0.3, 0.3333333], [16777216.0, 1.0, 3.0],
            [1e-30, 3e-30, 1e-29], [1e30, 1.0, 1e-30], [0.0])
    for n in range(1, 10):
        for m in (0, n, 3 * n):
            for k, vals in enumerate(sets):
                el = f32_edges(small.tiny_random(n, m, [1], seed=53 * n + m + k), vals, seed=n * 100 + m + k)
                adj = native.Adjacency(el.n, el.src, el.dst, el.w)
                c = graphgen.to_csr(el)
                g = sssp.Graph.from_csr(c, float_weights=True)
                for s in range(n):
                    if not model_completes(c, s):
                        skipped += 1
                        continue
                    d = g.solve(s).cpu().numpy()
                    assert sssp.counters()["flags"] == 0  # raises on an engine condition
                    assert_bits(d, adj.dijkstra_f32(s), "n=%d m=%d set=%d s=%d" % (n, m, k, s))
                    cases += 1
                g.close()
                adj.close()
    assert cases > 300 and skipped < 10, (cases, skipped)


def test_rounding_of_the_path_sum():
    # 0 -(2^24)- 1 -(1)- 2 -(1)- 3: each binary32 sum rounds to even, so
    # 2^24 + 1 = 2^24 and the distances of 1, 2, 3 are all 2^24; the direct
    # edge 0-3 of 2^24 + 4 is longer
    el = graphgen.from_arrays(4, [0, 1, 2, 0], [1, 2, 3, 3],
                              np.array([16777216.0, 1.0, 1.0, 16777220.0], np.float32).view(np.uint32))
    g = sssp.Graph.from_csr(graphgen.to_csr(el), float_weights=True)
    d = g.solve(0).cpu().numpy().view(np.float32)
    assert d.tolist() == [0.0, 16777216.0, 16777216.0, 16777216.0]


@pytest.mark.parametrize("topt", [True, False])
@pytest.mark.parametrize("name", ["rmat14f", "rmat14c1", "rmat14c5", "rmat14c9", "rmat16f"])
def test_real_weight_workloads(name, topt):
    wl = graphgen.workload(name)
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    g = sssp.Graph.from_csr(wl.csr, float_weights=True)
    pulls = 0
    for s in wl.sources(3):
        d = g.solve(int(s), traversal_opt=topt).cpu().numpy()
        c = sssp.counters()
        assert c["flags"] == 0
        pulls += c["pulls"]
        assert_bits(d, adj.dijkstra_f32(int(s)), "%s s=%d" % (name, s))
    # the ST_NUM grid gives the traversal optimisation a threshold below lb
    assert (pulls > 0) == topt
    adj.close()


@pytest.mark.parametrize("name", ["rmat12f", "rmat12c5", "rmat14f", "rmat14c9"])
def test_schedule_matches_the_f32_model(name):
    """<lb, ub, st> per step and the statistics taken at each step's end
    (sumD, highD, gap, the grid computeST) are functions of the settled set,
    so the GPU must reproduce the binary32 model step for step."""
    wl = graphgen.workload(name)
    c = wl.csr
    g = sssp.Graph.from_csr(c, float_weights=True)
    for s in wl.sources(3):
        ref = eic.eic_sssp_f32(c.n, c.rowptr, c.col, c.w, int(s))
        g.solve(int(s))
        got = sssp.schedule()
        assert len(got) == len(ref.steps), (len(got), len(ref.steps))
        for a, b in zip(got, ref.steps):
            assert (a["lb"], a["ub"], a["st"]) == (b.lb, b.ub, b.st), (a, b)
            if b.ub != INF or b.lb != 0:
                assert (a["L"], a["S"], a["h"], a["gap"], a["st_next"]) == \
                    (b.L, b.S, b.h, b.gap, b.st_next), (a, b)


def test_tree_and_point_to_point_with_real_weights():
    wl = graphgen.workload("rmat14c5")
    c = wl.csr
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    g = sssp.Graph.from_csr(c, float_weights=True)
    s = int(wl.sources(1)[0])
    ref = adj.dijkstra_f32(s)
    d, p = g.solve_tree(s)
    d = d.cpu().numpy()
    p = p.cpu().numpy()
    assert_bits(d, ref, "tree distances")
    assert p[s] == s
    df = d.view(np.float32)
    for v in np.nonzero((d != INF) & (np.arange(c.n) != s))[0][:2000]:
        u = int(p[v])
        lo, hi = c.rowptr[v], c.rowptr[v + 1]
        ws = c.w[lo:hi][c.col[lo:hi] == u].view(np.float32)
        assert any(np.float32(df[u]) + np.float32(x) == df[v] for x in ws), v
    assert np.all(p[d == INF] == -1)
    t = int(np.nonzero(ref != INF)[0][len(np.nonzero(ref != INF)[0]) // 2])
    dt, out = g.solve_p2p(s, t)
    assert dt == int(ref[t])
    low = ref <= dt
    assert np.array_equal(out.cpu().numpy()[low], ref[low])
    adj.close()


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -1.0, -0.0])
def test_invalid_real_weights_are_rejected(bad):
    el = graphgen.from_arrays(2, [0], [1], np.array([bad], np.float32).view(np.uint32))
    with pytest.raises(sssp.SSSPError):
        sssp.Graph.from_csr(graphgen.to_csr(el), float_weights=True)


def test_schedule_matches_the_f32_model_tiny_fuzz():
    sets = ([0.5, 0.25, 1.0], [0.1, 0.2, 0.7, 1e-3], [1e-30, 3e-30, 1e-29], [1e30, 1.0, 1e-30], [0.0])
    cases = 0
    for n in range(2, 10):
        for m in (n, 3 * n):
            for k, vals in enumerate(sets):
                el = f32_edges(small.tiny_random(n, m, [1], seed=71 * n + m + k), vals, seed=n * 31 + m + k)
                c = graphgen.to_csr(el)
                g = sssp.Graph.from_csr(c, float_weights=True)
                for s in range(n):
                    ref = eic.eic_sssp_f32(c.n, c.rowptr, c.col, c.w, s, max_steps=MODEL_STEPS)
                    if not ref.complete:
                        continue
                    steps = [b for b in ref.steps if not (b.lb == 0 and b.ub == INF)]
                    g.solve(s)
                    got = sssp.schedule()
                    assert len(got) == len(steps), (n, m, k, s)
                    for a, b in zip(got, steps):
                        assert (a["lb"], a["ub"], a["st"]) == (b.lb, b.ub, b.st), (n, m, k, s, a, b)
                    cases += 1
                g.close()
    assert cases > 150
