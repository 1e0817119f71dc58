"""GPU point-to-point queries (sssp_solve_p2p): the solve stops once the
target is settled. The target's distance is bit-exact with the oracle's, so
is the distance of every vertex the oracle puts at or below it, and every
other entry is an upper bound of its distance."""
import numpy as np
import pytest

import graphgen
from graphgen import small
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402

INF = 0xFFFFFFFF


def check_pair(g, ref, s, t):
    dt, out = g.solve_p2p(int(s), int(t))
    d = out.cpu().numpy()
    assert dt == int(ref[t]), (s, t, dt, int(ref[t]))
    # every vertex whose distance is not above the target's is settled by
    # then: the solve stops only once the band's lower end passes dt
    low = ref <= dt
    assert np.array_equal(d[low], ref[low]), (s, t)
    assert np.array_equal(d <= dt, low), (s, t)
    assert np.all(d.astype(np.uint64) >= ref.astype(np.uint64)), (s, t)
    c = sssp.counters()
    assert c["flags"] == 0
    return c


def test_tiny_fuzz_every_pair():
    cases = 0
    for n in range(1, 9):
        for m in (0, n, 3 * n):
            for weights in ([1], [1, 2, 3], [0, 1, 2]):
                el = small.tiny_random(n, m, weights, seed=311 * n + m + len(weights))
                g = sssp.Graph.from_csr(graphgen.to_csr(el))
                for s in range(n):
                    ref = native.dijkstra(el.n, el.src, el.dst, el.w, s)
                    for t in range(n):
                        check_pair(g, ref, s, t)
                        cases += 1
                g.close()
    assert cases > 500


@pytest.mark.parametrize("name", ["rmat14", "er16", "grid256"])
def test_workload_pairs_and_early_stop(name):
    wl = graphgen.workload(name)
    g = sssp.Graph.from_csr(wl.csr)
    rng = np.random.default_rng(5150)
    for s in wl.sources(2):
        s = int(s)
        ref = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, s)
        g.solve(s)
        full_steps = sssp.counters()["steps"]
        reach = np.nonzero(ref != INF)[0]
        # the nearest other vertex, a middle one and the farthest
        order = reach[np.argsort(ref[reach], kind="stable")]
        picks = [int(order[min(1, order.shape[0] - 1)]), int(order[order.shape[0] // 2]), int(order[-1])]
        picks += [int(x) for x in rng.choice(reach, size=3)]
        steps = []
        for t in picks:
            steps.append(check_pair(g, ref, s, t)["steps"])
        assert max(steps) <= full_steps
        assert steps[0] < full_steps or full_steps <= 2, (steps, full_steps)


def test_source_and_unreachable_targets():
    el = small.disjoint_union(small.path(5, [2, 2, 2, 2]), small.path(3, [1, 1]))
    g = sssp.Graph.from_csr(graphgen.to_csr(el))
    ref = native.dijkstra(el.n, el.src, el.dst, el.w, 0)
    c = check_pair(g, ref, 0, 0)
    assert c["steps"] <= 2
    dt, out = g.solve_p2p(0, 6)  # other component: unreachable, the whole solve runs
    assert dt == INF
    assert np.array_equal(out.cpu().numpy(), ref)


def test_target_out_of_range_is_rejected():
    wl = graphgen.workload("rmat12")
    g = sssp.Graph.from_csr(wl.csr)
    with pytest.raises(sssp.SSSPError):
        g.solve_p2p(0, wl.csr.n)
