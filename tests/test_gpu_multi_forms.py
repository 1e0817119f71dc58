"""Trees and point-to-point queries in the batched forms: k pairs in one launch
(sssp_solve_multi_ex), replayed plans (sssp_plan_create_ex / sssp_plan_run_ex)
and the query server (sssp_server_submit_ex). Full solves are bit-exact with
the Dijkstra oracle and their trees pass the oracle's tree checker; a
point-to-point pair is exact at its target and at every vertex whose distance
is not above the target's, an upper bound elsewhere, and its tree is tight on the
exact entries."""
import numpy as np
import pytest

import graphgen
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402

INF = 0xFFFFFFFF


def oracle(wl, s):
    return native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, int(s))


def check_full(wl, s, d, p=None):
    ref = oracle(wl, s)
    assert np.array_equal(d, ref), "distances differ (s=%d)" % s
    if p is not None:
        c = wl.csr
        assert native.check_tree(c.n, c.rowptr, c.col, c.w, int(s), d, p) == [0, 0, 0, 0], s
    return ref


def check_p2p(wl, s, t, d, p=None):
    ref = oracle(wl, s)
    dt = int(ref[t])
    assert int(d[t]) == dt
    low = ref <= dt
    assert np.array_equal(d[low], ref[low])
    assert np.array_equal(d <= dt, low)
    assert np.all(d.astype(np.uint64) >= ref.astype(np.uint64))
    if p is not None:
        c = wl.csr
        for v in np.nonzero(low & (ref != INF))[0][:3000]:
            v = int(v)
            u = int(p[v])
            if v == s:
                assert u == s
                continue
            lo, hi = c.rowptr[v], c.rowptr[v + 1]
            ws = c.w[lo:hi][c.col[lo:hi] == u]
            assert ws.shape[0] and int(ref[u]) + int(ws.min()) == int(ref[v]), (s, t, v, u)


def pick_target(ref, frac):
    reach = np.nonzero(ref != INF)[0]
    order = reach[np.argsort(ref[reach], kind="stable")]
    return int(order[int(frac * (order.shape[0] - 1))])


@pytest.mark.parametrize("trees", [False, True])
def test_multi_with_targets_and_trees(trees):
    wls = [graphgen.workload(n) for n in ("rmat14", "er12", "grid64", "rmat12")]
    gs = [sssp.Graph.from_csr(w.csr) for w in wls]
    srcs = [int(w.sources(1)[0]) for w in wls]
    # pairs 1 and 3 are point-to-point queries, 0 and 2 full solves
    tg = [-1, pick_target(oracle(wls[1], srcs[1]), 0.3), -1, pick_target(oracle(wls[3], srcs[3]), 0.6)]
    res = sssp.solve_multi(gs, srcs, targets=tg, trees=trees)
    outs, pars = res if trees else (res, [None] * 4)
    torch.cuda.synchronize()
    assert sssp.counters()["flags"] == 0
    for i, (w, s) in enumerate(zip(wls, srcs)):
        d = outs[i].cpu().numpy()
        p = None if pars[i] is None else pars[i].cpu().numpy()
        if tg[i] < 0:
            check_full(w, s, d, p)
        else:
            check_p2p(w, s, tg[i], d, p)
    for g in gs:
        g.close()


def test_multi_rejects_bad_targets():
    wl = graphgen.workload("rmat12")
    g = sssp.Graph.from_csr(wl.csr)
    with pytest.raises(sssp.SSSPError):
        sssp.solve_multi([g], [0], targets=[wl.csr.n])
    with pytest.raises(sssp.SSSPError):
        sssp.solve_multi([g], [0], targets=[-2])
    g.close()


def test_plan_with_trees_and_targets_replayed():
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    k = 4
    outs = [torch.empty(wl.csr.n, dtype=torch.uint32, device="cuda") for _ in range(k)]
    pars = [torch.empty(wl.csr.n, dtype=torch.int32, device="cuda") if i % 2 == 0 else None for i in range(k)]
    plan = sssp.Plan([g] * k, outs, parents=pars)
    srcs = [int(s) for s in wl.sources(2 * k)]
    for rep in range(2):
        ss = srcs[rep * k:(rep + 1) * k]
        tg = [-1] * k
        if rep == 1:
            tg[1] = pick_target(oracle(wl, ss[1]), 0.5)
            tg[2] = pick_target(oracle(wl, ss[2]), 0.2)
        plan.run(ss, targets=tg if rep == 1 else None)
        torch.cuda.synchronize()
        assert plan.counters()["flags"] == 0
        # eager work between replays
        g.solve(srcs[0])
        torch.cuda.synchronize()
        for i in range(k):
            d = outs[i].cpu().numpy()
            p = None if pars[i] is None else pars[i].cpu().numpy()
            if tg[i] < 0:
                check_full(wl, ss[i], d, p)
            else:
                check_p2p(wl, ss[i], tg[i], d, p)
    plan.close()
    g.close()


def test_server_tree_and_point_to_point_queries():
    wls = [graphgen.workload(n) for n in ("rmat14", "grid64")]
    gs = [sssp.Graph.from_csr(w.csr) for w in wls]
    srv = sssp.Server(budget_bytes=1 << 30, max_batch=4)
    ids = [srv.add_graph(g) for g in gs]
    jobs = []
    for rep in range(3):
        for gi, w in enumerate(wls):
            s = int(w.sources(3)[rep])
            out = torch.empty(w.csr.n, dtype=torch.uint32, device="cuda")
            kind = (rep + gi) % 3   # 0 plain, 1 tree, 2 point-to-point
            par = torch.empty(w.csr.n, dtype=torch.int32, device="cuda") if kind == 1 else None
            t = pick_target(oracle(w, s), 0.4) if kind == 2 else -1
            tk = srv.submit(ids[gi], s, out, target=t, parent=par)
            jobs.append((tk, gi, s, t, out, par))
    for tk, gi, s, t, out, par in jobs:
        srv.wait(tk)
        assert srv.info(tk)["status"] == 0
        d = out.cpu().numpy()
        p = None if par is None else par.cpu().numpy()
        if t < 0:
            check_full(wls[gi], s, d, p)
        else:
            check_p2p(wls[gi], s, t, d, p)
        srv.release(tk)
    srv.close()
    for g in gs:
        g.close()


def test_one_launch_mixing_weight_kinds_trees_and_targets():
    """Instances of one launch differ in weight kind (integer with the exact
    window, integer beyond it on the grid, binary32), in tree output and in
    point-to-point target; each must equal its own oracle."""
    names = ["rmat12", "rmat12f", "rmat12p20", "rmat12c5", "grid64w1000000", "er12"]
    wls = [graphgen.workload(n) for n in names]
    fl = [n.endswith("f") or "c" in n[4:] for n in names]
    gs = [sssp.Graph.from_csr(w.csr, float_weights=f) for w, f in zip(wls, fl)]
    srcs = [int(w.sources(1)[0]) for w in wls]
    adjs = [native.Adjacency(w.edges.n, w.edges.src, w.edges.dst, w.edges.w) for w in wls]
    refs = [a.dijkstra_f32(s) if f else a.dijkstra(s) for a, s, f in zip(adjs, srcs, fl)]
    tg = [-1, -1, pick_target(refs[2], 0.5), pick_target(refs[3], 0.3), -1, -1]
    outs, pars = sssp.solve_multi(gs, srcs, targets=tg, trees=True)
    torch.cuda.synchronize()
    assert sssp.counters()["flags"] == 0
    for i, w in enumerate(wls):
        d = outs[i].cpu().numpy()
        p = pars[i].cpu().numpy()
        ref = refs[i]
        if tg[i] < 0:
            assert np.array_equal(d, ref), names[i]
        else:
            dt = int(ref[tg[i]])
            assert int(d[tg[i]]) == dt, names[i]
            low = ref <= dt
            assert np.array_equal(d[low], ref[low]), names[i]
        # the parent of every exact, reachable vertex is joined to it by an edge
        # that is tight for the returned distances (binary32: in binary32)
        c = w.csr
        exact = (d == ref) & (ref != INF)
        if tg[i] >= 0:
            exact &= d <= int(ref[tg[i]])
        for v in np.nonzero(exact)[0][:1500]:
            v = int(v)
            u = int(p[v])
            if v == srcs[i]:
                assert u == v
                continue
            lo, hi = c.rowptr[v], c.rowptr[v + 1]
            ws = c.w[lo:hi][c.col[lo:hi] == u]
            assert ws.shape[0], (names[i], v, u)
            if fl[i]:
                du = np.array([ref[u]], np.uint32).view(np.float32)[0]
                ok = any(np.float32(du + np.array([x], np.uint32).view(np.float32)[0])
                         == np.array([ref[v]], np.uint32).view(np.float32)[0] for x in ws)
            else:
                ok = any(int(ref[u]) + int(x) == int(ref[v]) for x in ws)
            assert ok, (names[i], v, u)
    for a in adjs:
        a.close()
    for g in gs:
        g.close()
