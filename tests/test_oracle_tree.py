"""Pins for the predecessor part of the oracle (Section 2.1: the output of the
problem is the distance vector and, for every reachable vertex, its
predecessor on a shortest path): the Dijkstra tree against the definition
written out in Python on tiny graphs, trees that are unique by construction,
and planted mistakes the tree checker must catch."""
import numpy as np
import pytest

import graphgen
from graphgen import small
from oracle import native

INF = 0xFFFFFFFF

WEIGHT_SETS = {"unit": [1], "one_to_three": [1, 2, 3], "with_zero": [0, 1, 2], "zeros": [0, 0, 1]}


def tree_by_definition(n, src, dst, w, s, dist, parent):
    """True when parent is a shortest-path tree for dist, checked edge by edge
    on the raw undirected edge list: parent[s] = s; -1 exactly for the
    unreachable vertices; every other parent is joined to its child by an edge
    with dist[p] + w = dist[v]; following parents from any reachable vertex
    reaches s within n steps."""
    dist = [int(x) for x in dist]
    parent = [int(x) for x in parent]
    if parent[s] != s:
        return False
    edges = list(zip(src.tolist(), dst.tolist(), w.tolist()))
    for v in range(n):
        if dist[v] == INF:
            if parent[v] != -1:
                return False
            continue
        if v == s:
            continue
        p = parent[v]
        if not 0 <= p < n or dist[p] == INF:
            return False
        if not any({a, b} == {p, v} and dist[p] + c == dist[v] for a, b, c in edges):
            return False
        x, steps = v, 0
        while x != s:
            x = parent[x]
            steps += 1
            if steps > n or x < 0:
                return False
    return True


@pytest.mark.parametrize("wname", sorted(WEIGHT_SETS))
def test_dijkstra_tree_matches_the_definition_tiny_fuzz(wname):
    weights = WEIGHT_SETS[wname]
    for n in range(1, 11):
        for m in (0, n, 2 * n, 3 * n):
            el = small.tiny_random(n, m, weights, seed=7000 + 100 * n + m)
            adj = native.Adjacency(n, el.src, el.dst, el.w)
            csr = graphgen.to_csr(el)
            for s in range(n):
                d, par = adj.dijkstra_tree(s)
                assert np.array_equal(d, adj.dijkstra(s))
                assert tree_by_definition(n, el.src, el.dst, el.w, s, d, par), (n, m, s)
                assert native.check_tree(n, csr.rowptr, csr.col, csr.w, s, d, par) == [0, 0, 0, 0]


def test_unique_trees():
    # a path: the only tree is the path itself
    el = small.path(6, [3, 1, 4, 1, 5])
    adj = native.Adjacency(el.n, el.src, el.dst, el.w)
    d, par = adj.dijkstra_tree(0)
    assert d.tolist() == [0, 3, 4, 8, 9, 14]
    assert par.tolist() == [0, 0, 1, 2, 3, 4]
    d, par = adj.dijkstra_tree(3)
    assert par.tolist() == [1, 2, 3, 3, 3, 4]
    # a star with an unreachable extra vertex
    el = small.disjoint_union(small.star(4, [2, 7, 1, 8]), small.path(1, []))
    adj = native.Adjacency(el.n, el.src, el.dst, el.w)
    d, par = adj.dijkstra_tree(2)
    assert d.tolist() == [7, 9, 0, 8, 15, INF]
    assert par.tolist() == [2, 0, 2, 0, 0, -1]


def _planted_case():
    # 0 -1- 1 -0- 2 -0- 3, 1 -5- 4, and 5 isolated (unreachable); source 0
    el = graphgen.from_arrays(6, [0, 1, 2, 1], [1, 2, 3, 4], [1, 0, 0, 5])
    csr = graphgen.to_csr(el)
    adj = native.Adjacency(el.n, el.src, el.dst, el.w)
    d, par = adj.dijkstra_tree(0)
    assert d.tolist() == [0, 1, 1, 1, 6, INF]
    assert par.tolist() == [0, 0, 1, 2, 1, -1]
    return el, csr, d, par


@pytest.mark.parametrize("mistake, slot", [
    ("source_parent", 0),   # parent[s] = 1
    ("unreachable_has_parent", 1),   # parent[5] = 4
    ("not_a_vertex", 1),    # parent[4] = 17
    ("not_adjacent", 2),    # parent[4] = 0: no edge 0-4
    ("not_tight", 2),       # parent[4] = 1 with dist[4] lowered by one
    ("zero_weight_cycle", 3),   # parent[2] = 3, parent[3] = 2 (both edges tight)
])
def test_tree_checker_catches_planted_mistakes(mistake, slot):
    el, csr, d, par = _planted_case()
    d = d.copy()
    par = par.copy()
    if mistake == "source_parent":
        par[0] = 1
    elif mistake == "unreachable_has_parent":
        par[5] = 4
    elif mistake == "not_a_vertex":
        par[4] = 17
    elif mistake == "not_adjacent":
        par[4] = 0
    elif mistake == "not_tight":
        d[4] = 5
    elif mistake == "zero_weight_cycle":
        par[2] = 3
        par[3] = 2
    counts = native.check_tree(el.n, csr.rowptr, csr.col, csr.w, 0, d, par)
    assert counts[slot] > 0, (mistake, counts)
    assert not tree_by_definition(el.n, el.src, el.dst, el.w, 0, d, par)


def test_tree_checker_accepts_other_valid_trees():
    # ties: both 0-1-3 and 0-2-3 are shortest; either parent of 3 is valid
    el = graphgen.from_arrays(4, [0, 0, 1, 2], [1, 2, 3, 3], [1, 1, 1, 1])
    csr = graphgen.to_csr(el)
    d = np.array([0, 1, 1, 2], np.uint32)
    for p3 in (1, 2):
        par = np.array([0, 0, 0, p3], np.int32)
        assert native.check_tree(4, csr.rowptr, csr.col, csr.w, 0, d, par) == [0, 0, 0, 0]
        assert tree_by_definition(4, el.src, el.dst, el.w, 0, d, par)
