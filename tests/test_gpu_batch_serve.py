"""GPU: the batched forms -- graph-captured plans, the autotuner and the
query server -- give the same distances as the oracle (and as plain solves),
whatever runs beside a query. All calls go through the C ABI."""
import time

import numpy as np
import pytest

import graphgen
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402


def oracle_dist(el, s):
    return native.dijkstra(el.n, el.src, el.dst, el.w, int(s))


def same(a, b, what):
    if not np.array_equal(a, b):
        bad = np.nonzero(a != b)[0]
        raise AssertionError("%s: %d differ, first %s" % (what, bad.shape[0], bad[:5]))


def test_plan_replays_one_graph():
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    k = 8
    outs = [torch.empty(wl.csr.n, dtype=torch.uint32, device="cuda") for _ in range(k)]
    plan = sssp.Plan([g] * k, outs)
    srcs = [int(s) for s in wl.sources(3 * k)]
    for rep in range(3):
        batch = srcs[rep * k:(rep + 1) * k]
        plan.run(batch)
        torch.cuda.synchronize()
        assert plan.counters()["flags"] == 0
        for i, s in enumerate(batch):
            same(outs[i].cpu().numpy(), oracle_dist(wl.edges, s), "replay %d row %d" % (rep, i))
        # eager work between replays
        g.solve(srcs[0])
        torch.cuda.synchronize()
    plan.close()


def test_plan_replays_many_graphs():
    wls = [graphgen.workload(n) for n in ("rmat10", "rmat11", "rmat12", "rmat13", "grid40", "er10")]
    gs = [sssp.Graph.from_csr(w.csr) for w in wls]
    outs = [torch.empty(w.csr.n, dtype=torch.uint32, device="cuda") for w in wls]
    plan = sssp.Plan(gs, outs)
    for rep in range(2):
        srcs = [int(w.sources(2)[rep]) for w in wls]
        plan.run(srcs)
        torch.cuda.synchronize()
        for w, s, o in zip(wls, srcs, outs):
            same(o.cpu().numpy(), oracle_dist(w.edges, s), "%s replay %d" % (w.name, rep))
    plan.close()


def test_autotune_changes_no_distance():
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    srcs = [int(s) for s in wl.sources(3)]
    tuned, rep = sssp.autotune([g] * 3, srcs, tune_beta=True)
    assert rep["evaluations"] >= 4 and rep["best_us"] <= rep["default_us"]
    for s in srcs:
        same(g.solve(s, **tuned).cpu().numpy(), oracle_dist(wl.edges, s), "tuned s=%d" % s)
    tuned_b, rep_b = sssp.autotune([g] * 3, srcs, batched=True)
    out = sssp.solve_multi([g] * 3, srcs, **tuned_b)
    for s, o in zip(srcs, out):
        same(o.cpu().numpy(), oracle_dist(wl.edges, s), "tuned batch s=%d" % s)


def _mix():
    wls = [graphgen.workload(n) for n in ("rmat12", "rmat14", "grid64", "er12")]
    return wls, [sssp.Graph.from_csr(w.csr) for w in wls]


def test_server_alone_and_in_the_mix_agree():
    wls, gs = _mix()
    rng = np.random.default_rng(5)
    queries = []
    for q in range(40):
        gi = int(rng.integers(0, len(wls)))
        queries.append((gi, int(wls[gi].sources(8)[q % 8])))
    alone = [gs[gi].solve(s).cpu().numpy() for gi, s in queries]
    srv = sssp.Server(budget_bytes=8 << 30, max_batch=8, ticks_per_launch=4)
    ids = [srv.add_graph(g) for g in gs]
    outs = [torch.empty(wls[gi].csr.n, dtype=torch.uint32, device="cuda") for gi, _ in queries]
    tickets = []
    for qi, (gi, s) in enumerate(queries):
        tickets.append(srv.submit(ids[gi], s, outs[qi]))
        if qi % 5 == 4:
            time.sleep(0.002)  # later queries arrive while earlier ones run
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    assert st["completed"] == len(queries) and st["launches"] > 1 and st["peak_active"] > 1
    for qi, (gi, s) in enumerate(queries):
        same(outs[qi].cpu().numpy(), alone[qi], "query %d (graph %d, s=%d)" % (qi, gi, s))
        info = srv.info(tickets[qi])
        assert info["state"] == 0 and info["status"] == 0
        assert info["submit_us"] <= info["admit_us"] <= info["done_us"]
    for qi in (0, 7, 23):
        gi, s = queries[qi]
        same(outs[qi].cpu().numpy(), oracle_dist(wls[gi].edges, s), "oracle %d" % qi)
    srv.close()


def test_server_admission_by_budget():
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    srv = sssp.Server(budget_bytes=1 << 40, max_batch=16, ticks_per_launch=2)
    gid = srv.add_graph(g)
    qb = srv.query_bytes(gid)
    srv.close()
    srv = sssp.Server(budget_bytes=int(2.5 * qb), max_batch=16, ticks_per_launch=2)
    gid = srv.add_graph(g)
    srcs = [int(s) for s in wl.sources(12)]
    outs = [torch.empty(wl.csr.n, dtype=torch.uint32, device="cuda") for _ in srcs]
    tickets = [srv.submit(gid, s, o) for s, o in zip(srcs, outs)]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    assert 1 <= st["peak_active"] <= 2, st
    assert st["peak_in_use_bytes"] <= int(2.5 * qb)
    for s, o in zip(srcs, outs):
        same(o.cpu().numpy(), oracle_dist(wl.edges, s), "budgeted s=%d" % s)
    srv.close()
    small = sssp.Server(budget_bytes=qb // 2, max_batch=4)
    gid = small.add_graph(g)
    with pytest.raises(sssp.SSSPError) as ei:
        small.submit(gid, srcs[0], outs[0])
    assert ei.value.status == -3
    with pytest.raises(sssp.SSSPError):
        small.submit(gid + 5, srcs[0], outs[0])
    with pytest.raises(sssp.SSSPError):
        small.submit(gid, wl.csr.n, outs[0])
    small.close()


def test_server_tree_queries_within_the_budget():
    """A tree query counts its parent output and the solve's 8-byte tree words
    against the budget: with room for a little more than one tree query, tree
    and plain queries still all complete, correct, and the memory in use never
    exceeds the budget; a budget too small for a tree query (but large enough
    for a plain one) rejects it at submission."""
    from oracle import native
    wl = graphgen.workload("rmat14")
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    srv = sssp.Server(budget_bytes=1 << 40, max_batch=8, ticks_per_launch=2)
    gid = srv.add_graph(g)
    qb = srv.query_bytes(gid)
    srv.close()
    tree_b = qb + 12 * c.n
    budget = int(1.3 * tree_b)
    srv = sssp.Server(budget_bytes=budget, max_batch=8, ticks_per_launch=2)
    gid = srv.add_graph(g)
    srcs = [int(s) for s in wl.sources(6)]
    outs = [torch.empty(c.n, dtype=torch.uint32, device="cuda") for _ in srcs]
    pars = [torch.empty(c.n, dtype=torch.int32, device="cuda") if i % 2 == 0 else None for i in range(len(srcs))]
    tickets = [srv.submit(gid, s, o, parent=p) for s, o, p in zip(srcs, outs, pars)]
    for t in tickets:
        srv.wait(t)
        assert srv.info(t)["status"] == 0
    st = srv.stats()
    assert st["completed"] == len(srcs)
    assert st["peak_in_use_bytes"] <= budget, st
    for s, o, p in zip(srcs, outs, pars):
        d = o.cpu().numpy()
        same(d, oracle_dist(wl.edges, s), "tree-budget s=%d" % s)
        if p is not None:
            assert native.check_tree(c.n, c.rowptr, c.col, c.w, s, d, p.cpu().numpy()) == [0, 0, 0, 0]
    srv.close()
    tight = sssp.Server(budget_bytes=qb + 4 * c.n, max_batch=2)
    gid = tight.add_graph(g)
    with pytest.raises(sssp.SSSPError) as ei:
        tight.submit(gid, srcs[0], outs[0], parent=pars[0])
    assert ei.value.status == -3
    t = tight.submit(gid, srcs[1], outs[1])
    tight.wait(t)
    same(outs[1].cpu().numpy(), oracle_dist(wl.edges, srcs[1]), "plain in a tight budget")
    tight.close()
    g.close()
