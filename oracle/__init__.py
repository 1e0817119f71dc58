"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU statement of what the GPU engine computes,
written from the paper (Yu, Wang, Luo, "A Heuristic Algorithm for Shortest
Path Search"):

* ``native``    (``dijkstra.c``) single-source shortest paths by definition:
  binary-heap Dijkstra over the raw undirected edge list (Section 2's problem
  statement; Dijkstra as in Section 2.2), plus an invariant checker.
* ``heuristic`` the statistics and Eq. (1)-(6), RtoW[] and computeST
  (Sections 3.1, 3.2, 3.3, 4.1).
* ``eic``       a sequential model of the whole heuristic algorithm (the
  Algorithm with Functions 1 and 2) that yields the per-step schedule.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import anything from here. The GPU library shares no code with it.

Pins (what ties each function to something other than itself) live in
``tests/test_oracle_*.py``: brute force (Bellman-Ford, Floyd-Warshall, an
exhaustive threshold search for highD), closed forms (BFS hop counts, path
prefix sums, grid Manhattan distances), the paper's own numbers (Table 1's
highD(0) of a uniform-random graph and of the scale-26 R-MAT graphs), the
quantile definition of maxW and the identity (1 - ratio)^(prob * highD) =
1 - prob behind Eq. (2).  computeST's profit estimate has no printed value to
check against; its guards, its clamps and a hand-worked window are pinned.
"""
