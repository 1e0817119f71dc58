"""GPU shortest-path trees (sssp_solve_tree): distances bit-exact with the
Dijkstra oracle and the predecessor array valid for them (the oracle's tree
checker: parent[s] = s, -1 exactly where unreachable, every parent edge tight,
every chain ending at s). Several trees are correct when shortest paths tie,
so the parents are checked for validity, not compared entry by entry, except
where the tree is unique."""
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


def check(el, csr, g, s, **opts):
    d, p = g.solve_tree(int(s), **opts)
    d = d.cpu().numpy()
    p = p.cpu().numpy()
    ref = native.dijkstra(el.n, el.src, el.dst, el.w, int(s))
    assert np.array_equal(d, ref), "distances differ from the oracle (s=%d)" % s
    counts = native.check_tree(csr.n, csr.rowptr, csr.col, csr.w, int(s), d, p)
    assert counts == [0, 0, 0, 0], (s, counts)
    c = sssp.counters()
    assert c["flags"] == 0
    return d, p


def test_tiny_fuzz_trees_with_zero_weights():
    cases = 0
    for n in range(1, 11):
        for m in (0, n, 3 * n):
            for weights in ([1], [1, 2, 3], [0, 1, 2], [0, 0, 1]):
                el = small.tiny_random(n, m, weights, seed=977 * n + m + len(weights))
                csr = graphgen.to_csr(el)
                g = sssp.Graph.from_csr(csr)
                for s in range(n):
                    check(el, csr, g, s)
                    cases += 1
                g.close()
    assert cases > 300


def test_unique_tree_of_a_path():
    el = small.path(6, [3, 1, 4, 1, 5])
    csr = graphgen.to_csr(el)
    g = sssp.Graph.from_csr(csr)
    _, p = check(el, csr, g, 3)
    assert p.tolist() == [1, 2, 3, 3, 3, 4]


@pytest.mark.parametrize("name", ["rmat14", "er16", "grid256"])
@pytest.mark.parametrize("topt", [True, False])
def test_workload_trees(name, topt):
    wl = graphgen.workload(name)
    g = sssp.Graph.from_csr(wl.csr)
    for s in wl.sources(3):
        check(wl.edges, wl.csr, g, s, traversal_opt=topt)


def test_zero_weight_plateaus():
    # a lattice whose weights are mostly 0: large equal-distance plateaus, where
    # only the order in which vertices reached their distance prevents cycles
    rng = np.random.default_rng(20250630)
    el = small.lattice(48, 48, 1)
    w = rng.choice(np.array([0, 0, 0, 1, 2], dtype=np.uint32), size=el.src.shape[0])
    el = graphgen.from_arrays(el.n, el.src, el.dst, w)
    csr = graphgen.to_csr(el)
    g = sssp.Graph.from_csr(csr)
    for s in (0, 1000, 2303):
        check(el, csr, g, s)


def test_tree_solve_leaves_distances_unchanged():
    wl = graphgen.workload("rmat14")
    g = sssp.Graph.from_csr(wl.csr)
    for s in wl.sources(2):
        plain = g.solve(int(s)).cpu().numpy()
        d, _ = g.solve_tree(int(s))
        assert np.array_equal(plain, d.cpu().numpy())
        # and a plain solve after a tree solve on the same stream
        assert np.array_equal(plain, g.solve(int(s)).cpu().numpy())
