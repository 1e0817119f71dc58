"""GPU parity at the full sizes of the measured workloads, in the launch
configuration bench.py times: RMAT-24 (every distance checked by the
oracle's invariant checker, which characterises them completely for weights
>= 1; bench.py compares one source with the oracle's Dijkstra; a
shortest-path tree checked by the oracle's tree checker), RMAT-24 with real
binary32 weights against the oracle's binary32 Dijkstra, ER-22 and the
2048 x 2048 grid against the oracle's Dijkstra, and the 64-source RMAT-22
plan (sampled rows)."""
import numpy as np
import pytest

import graphgen
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402


def assert_same(got, ref, what):
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError("%s: %d of %d differ; first %s" % (what, bad.shape[0], got.shape[0], bad[:5]))


def invariant_ok(c, s, d):
    return sum(native.check_sssp(c.n, c.rowptr, c.col, c.w, int(s), d)) == 0


def test_rmat24_invariants():
    wl = graphgen.workload("rmat24")
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    srcs = [int(s) for s in wl.sources(3)]
    outs = []
    for s in srcs:
        outs.append(g.solve(s).cpu().numpy())
        assert sssp.counters()["flags"] == 0
    for s, d in zip(srcs, outs):
        assert d[s] == 0 and invariant_ok(c, s, d), "rmat24 s=%d" % s
    # filter off: the same distances
    d_off = g.solve(srcs[0], traversal_opt=False).cpu().numpy()
    assert_same(d_off, outs[0], "rmat24 filter off")
    g.close()


def test_rmat24_tree():
    # a shortest-path tree at full size: the same distances as the plain solve,
    # and a valid predecessor array for them (the oracle's tree checker)
    wl = graphgen.workload("rmat24")
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    s = int(wl.sources(1)[0])
    plain = g.solve(s).cpu().numpy()
    d, p = g.solve_tree(s)
    assert sssp.counters()["flags"] == 0
    d = d.cpu().numpy()
    assert_same(d, plain, "rmat24 tree distances")
    assert invariant_ok(c, s, d)
    assert native.check_tree(c.n, c.rowptr, c.col, c.w, s, d, p.cpu().numpy()) == [0, 0, 0, 0]
    g.close()


def test_rmat24_real_weights():
    # weights uniform on (0, 1]: one source against the oracle's binary32
    # Dijkstra, with the traversal optimisation on (the ST_NUM grid) and off
    wl = graphgen.workload("rmat24f")
    c = wl.csr
    g = sssp.Graph.from_csr(c, float_weights=True)
    s = int(wl.sources(1)[0])
    on = g.solve(s).cpu().numpy()
    cnt = sssp.counters()
    assert cnt["flags"] == 0 and cnt["pulls"] > 0
    off = g.solve(s, traversal_opt=False).cpu().numpy()
    assert sssp.counters()["flags"] == 0
    g.close()
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    ref = adj.dijkstra_f32(s)
    adj.close()
    assert_same(on, ref, "rmat24f")
    assert_same(off, ref, "rmat24f filter off")


def test_er22_against_oracle():
    wl = graphgen.workload("er22")
    g = sssp.Graph.from_csr(wl.csr)
    srcs = [int(s) for s in wl.sources(8)]
    outs = [g.solve(s).cpu().numpy() for s in srcs]
    assert sssp.counters()["flags"] == 0
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    refs = adj.dijkstra_many(srcs[:4], 8)
    adj.close()
    for i in range(4):
        assert_same(outs[i], refs[i], "er22 s=%d" % srcs[i])
    for s, d in zip(srcs[4:], outs[4:]):
        assert invariant_ok(wl.csr, s, d), "er22 invariants s=%d" % s


def test_grid2048_against_oracle():
    wl = graphgen.workload("grid2048")
    g = sssp.Graph.from_csr(wl.csr)
    srcs = [int(s) for s in wl.sources(2)]
    outs = [g.solve(s).cpu().numpy() for s in srcs]
    assert sssp.counters()["flags"] == 0
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    refs = adj.dijkstra_many(srcs, 2)
    adj.close()
    for s, d, r in zip(srcs, outs, refs):
        assert_same(d, r, "grid2048 s=%d" % s)


def test_rmat22_64_source_plan_rows():
    wl = graphgen.workload("rmat22")
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    k = 64
    srcs = [int(s) for s in wl.sources(k)]
    outs = [torch.empty(c.n, dtype=torch.uint32, device="cuda") for _ in range(k)]
    plan = sssp.Plan([g] * k, outs)
    plan.run(srcs)
    torch.cuda.synchronize()
    assert plan.counters()["flags"] == 0
    for i in (0, 17, 40, 63):
        assert invariant_ok(c, srcs[i], outs[i].cpu().numpy()), "rmat22 plan row %d" % i
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    ref = adj.dijkstra(srcs[5])
    adj.close()
    assert_same(outs[5].cpu().numpy(), ref, "rmat22 plan row 5 vs oracle")
    plan.close()
