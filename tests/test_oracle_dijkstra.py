"""Pins for the Dijkstra oracle: brute force on tiny graphs, closed forms,
hand-worked fixtures, multigraph semantics and the invariant checker."""
import collections
import itertools

import numpy as np
import pytest

import graphgen
from graphgen import small
from oracle import native

from _fixtures import INF, all_fixtures

WEIGHT_SETS = {
    "unit": [1],
    "one_to_three": [1, 2, 3],
    "byte": list(range(1, 256)),
    "with_zero": [0, 1, 2, 3],
}


def bellman_ford(n, src, dst, w, s):
    """|V|-1 rounds of relaxing every edge both ways (Section 2.2's Bellman-Ford)."""
    d = [None] * n
    d[s] = 0
    for _ in range(max(n - 1, 1)):
        changed = False
        for u, v, c in zip(src.tolist(), dst.tolist(), w.tolist()):
            for a, b in ((u, v), (v, u)):
                if d[a] is not None and (d[b] is None or d[a] + c < d[b]):
                    d[b] = d[a] + c
                    changed = True
        if not changed:
            break
    return np.array([INF if x is None else x for x in d], dtype=np.uint64).astype(np.uint32)


def floyd_warshall(n, src, dst, w):
    big = np.iinfo(np.int64).max // 4
    D = np.full((n, n), big, dtype=np.int64)
    np.fill_diagonal(D, 0)
    for u, v, c in zip(src.tolist(), dst.tolist(), w.tolist()):
        D[u, v] = min(D[u, v], c)
        D[v, u] = min(D[v, u], c)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    D[D >= big] = INF
    return D


@pytest.mark.parametrize("wname", sorted(WEIGHT_SETS))
def test_dijkstra_matches_bellman_ford_tiny_fuzz(wname):
    weights = WEIGHT_SETS[wname]
    cases = 0
    for n in range(1, 13):
        for m in (0, n // 2, n, 2 * n, 3 * n):
            for rep in range(3):
                el = small.tiny_random(n, m, weights, seed=1000 * n + 10 * m + rep)
                for s in range(n):
                    got = native.dijkstra(el.n, el.src, el.dst, el.w, s)
                    ref = bellman_ford(el.n, el.src, el.dst, el.w, s)
                    assert np.array_equal(got, ref), (n, m, rep, s)
                    cases += 1
    assert cases > 1000


def test_dijkstra_matches_floyd_warshall():
    for seed in range(20):
        n = 9 + seed % 5
        el = small.tiny_random(n, 3 * n, list(range(0, 50)), seed=seed)
        D = floyd_warshall(n, el.src, el.dst, el.w)
        for s in range(n):
            got = native.dijkstra(el.n, el.src, el.dst, el.w, s)
            assert np.array_equal(got, D[s].astype(np.uint32)), (seed, s)


def _bfs_hops(n, src, dst, s):
    adj = collections.defaultdict(list)
    for u, v in zip(src.tolist(), dst.tolist()):
        adj[u].append(v)
        adj[v].append(u)
    d = [INF] * n
    d[s] = 0
    q = collections.deque([s])
    while q:
        u = q.popleft()
        for v in adj[u]:
            if d[v] == INF:
                d[v] = d[u] + 1
                q.append(v)
    return np.array(d, dtype=np.uint32)


def test_unit_weights_are_bfs_hops():
    for seed in range(5):
        el = graphgen.gnm(2000, 3000, wmax=1, seed=seed)
        for s in (0, 7, 1999):
            got = native.dijkstra(el.n, el.src, el.dst, el.w, s)
            assert np.array_equal(got, _bfs_hops(el.n, el.src, el.dst, s))


def test_path_is_prefix_sums():
    rng = np.random.default_rng(3)
    w = rng.integers(0, 1000, size=499)
    el = small.path(500, w)
    got = native.dijkstra(el.n, el.src, el.dst, el.w, 0)
    assert np.array_equal(got.astype(np.int64), np.concatenate([[0], np.cumsum(w)]))
    mid = 250
    got = native.dijkstra(el.n, el.src, el.dst, el.w, mid)
    pre = np.concatenate([[0], np.cumsum(w)])
    assert np.array_equal(got.astype(np.int64), np.abs(pre - pre[mid]))


def test_lattice_is_scaled_manhattan():
    rows, cols, c = 31, 47, 7
    el = small.lattice(rows, cols, c)
    s = 5 * cols + 11
    got = native.dijkstra(el.n, el.src, el.dst, el.w, s).reshape(rows, cols).astype(np.int64)
    r, k = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    assert np.array_equal(got, c * (np.abs(r - 5) + np.abs(k - 11)))


def test_star_and_components():
    el = small.disjoint_union(small.star(50, np.arange(1, 51)), small.lattice(3, 3, 2))
    got = native.dijkstra(el.n, el.src, el.dst, el.w, 0)
    assert got[0] == 0 and np.array_equal(got[1:51], np.arange(1, 51))
    assert np.all(got[51:] == INF)
    got = native.dijkstra(el.n, el.src, el.dst, el.w, 7)  # a leaf: via the hub
    assert got[0] == 7 and got[3] == 10 and got[7] == 0


@pytest.mark.parametrize("fx", all_fixtures(), ids=lambda f: f["name"])
def test_golden_fixtures(fx):
    if fx["overflow"]:
        with pytest.raises(OverflowError):
            native.dijkstra(fx["n"], fx["src"], fx["dst"], fx["w"], fx["s"])
        return
    got = native.dijkstra(fx["n"], fx["src"], fx["dst"], fx["w"], fx["s"])
    assert np.array_equal(got, fx["dist"])


def test_raw_multigraph_equals_cleaned_csr():
    """Dropping self-loops and merging parallel edges to their minimum weight
    (the CSR cleaning) must not change any distance."""
    for seed in range(10):
        el = small.tiny_random(40, 200, list(range(0, 20)), seed=seed)
        csr = graphgen.to_csr(el)
        rows = np.repeat(np.arange(csr.n), np.diff(csr.rowptr))
        for s in (0, 13, 39):
            a = native.dijkstra(el.n, el.src, el.dst, el.w, s)
            b = native.dijkstra(csr.n, rows, csr.col, csr.w, s)
            assert np.array_equal(a, b)


def _csr_of(el):
    return graphgen.to_csr(el)


def test_checker_accepts_exact_and_rejects_planted_mistakes():
    wl = graphgen.workload("rmat12")
    c = wl.csr
    s = int(wl.sources(1)[0])
    d = native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w, s)
    assert native.check_sssp(c.n, c.rowptr, c.col, c.w, s, d) == [0, 0, 0, 0, 0]
    reach = np.nonzero((d != INF) & (np.arange(c.n) != s))[0]
    v = int(reach[len(reach) // 2])
    bad = d.copy(); bad[v] += 1          # too long: some edge improves it
    assert native.check_sssp(c.n, c.rowptr, c.col, c.w, s, bad)[1] > 0
    bad = d.copy(); bad[v] -= 1          # too short: no tight in-edge
    assert native.check_sssp(c.n, c.rowptr, c.col, c.w, s, bad)[2] > 0
    bad = d.copy(); bad[s] = 1
    assert native.check_sssp(c.n, c.rowptr, c.col, c.w, s, bad)[0] > 0
    bad = d.copy(); bad[v] = INF         # reachable vertex reported unreachable
    assert sum(native.check_sssp(c.n, c.rowptr, c.col, c.w, s, bad)) > 0


def test_checker_closes_zero_weight_loophole():
    """Two vertices joined by a zero edge can vouch for each other at a wrong
    value; only the tight-reachability check from s catches it."""
    el = graphgen.from_arrays(4, [0, 1, 2], [1, 2, 3], [5, 0, 4])
    c = _csr_of(el)
    good = native.dijkstra(el.n, el.src, el.dst, el.w, 0)
    assert list(good) == [0, 5, 5, 9]
    assert native.check_sssp(c.n, c.rowptr, c.col, c.w, 0, good) == [0, 0, 0, 0, 0]
    # a disconnected zero-weight pair claiming a finite distance
    el2 = graphgen.from_arrays(4, [0, 2], [1, 3], [5, 0])
    c2 = _csr_of(el2)
    bad = np.array([0, 5, 9, 9], dtype=np.uint32)
    counts = native.check_sssp(c2.n, c2.rowptr, c2.col, c2.w, 0, bad)
    assert counts[2] == 0 and counts[3] == 2


def test_many_sources_threaded_equals_single():
    wl = graphgen.workload("rmat11")
    srcs = wl.sources(12)
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    many = adj.dijkstra_many(srcs, threads=4)
    for i, s in enumerate(srcs):
        assert np.array_equal(many[i], adj.dijkstra(int(s)))
    adj.close()
