"""The seeded input generators: determinism, shapes, and the CSR cleaning rule."""
import hashlib

import numpy as np
import pytest

import graphgen
from graphgen import small


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def test_generators_are_deterministic_and_seeded():
    for make in (lambda s: graphgen.rmat(10, 16, seed=s), lambda s: graphgen.gnm(1000, 8000, seed=s),
                 lambda s: graphgen.grid(30, 40, seed=s)):
        a, b, c = make(1), make(1), make(2)
        assert _digest(a.src, a.dst, a.w) == _digest(b.src, b.dst, b.w)
        assert _digest(a.src, a.dst, a.w) != _digest(c.src, c.dst, c.w)


def test_rmat14_shape():
    wl = graphgen.workload("rmat14")
    el, c = wl.edges, wl.csr
    assert el.n == 16384 and el.m == 16 * 16384
    assert el.w.min() >= 1 and el.w.max() <= 255
    deg = c.degrees()
    # about 262K generated edges -> ~213K after cleaning; ~23% isolated
    assert 200_000 < c.nnz // 2 < 230_000
    assert 0.15 < (deg == 0).mean() < 0.3


def test_weights_uniform():
    el = graphgen.gnm(1 << 12, 1 << 18, wmax=255, seed=3)
    counts = np.bincount(el.w, minlength=256)[1:]
    assert counts.min() > 0.8 * counts.mean() and counts.max() < 1.2 * counts.mean()


def test_csr_cleaning_rule():
    """Self-loops dropped, both directions stored, one entry per neighbour
    carrying the minimum weight of the parallel edges, rows sorted by column."""
    el = small.tiny_random(50, 400, list(range(0, 30)), seed=4)
    c = graphgen.to_csr(el)
    best = {}
    for u, v, w in zip(el.src.tolist(), el.dst.tolist(), el.w.tolist()):
        if u == v:
            continue
        for a, b in ((u, v), (v, u)):
            best[(a, b)] = min(best.get((a, b), 1 << 40), w)
    got = {}
    for u in range(c.n):
        cols = c.col[c.rowptr[u]:c.rowptr[u + 1]]
        assert np.all(np.diff(cols) > 0)
        for v, w in zip(cols.tolist(), c.w[c.rowptr[u]:c.rowptr[u + 1]].tolist()):
            got[(u, v)] = w
    assert got == best


def test_grid_structure():
    el = graphgen.grid(64, 64, p_keep=0.95, p_diag=0.01, wmax=1000, seed=9)
    c = graphgen.to_csr(el)
    deg = c.degrees()
    assert deg.max() <= 6
    assert 0.93 < (c.nnz / 2) / (2 * 64 * 63) < 0.99 + 0.01
    assert el.w.min() >= 1 and el.w.max() <= 1000
    r, k = el.src // 64, el.src % 64
    r2, k2 = el.dst // 64, el.dst % 64
    dr, dk = r2 - r, k2 - k
    assert set(zip(dr.tolist(), dk.tolist())) <= {(0, 1), (1, 0), (1, 1)}


def test_sources_have_edges_and_are_distinct():
    wl = graphgen.workload("rmat12")
    srcs = wl.sources(64)
    deg = wl.csr.degrees()
    assert len(set(srcs.tolist())) == 64
    assert np.all(deg[srcs] >= 1)
    assert np.array_equal(srcs, wl.sources(64))


@pytest.mark.parametrize("power", [1, 2, 3, 4, 6, 8, 10])
def test_integer_power_weights(power):
    """Eq. 7's variant weights: exactly the 2^power - 1 integers 1 .. 2^power - 1,
    the inner ones equally likely and the two ends half as likely (the nearest
    integer to 1 + x (2^power - 2), x uniform on (0, 1]); repeatable."""
    m = 400000
    w = graphgen.weights_power(m, power, 4242)
    assert np.array_equal(w, graphgen.weights_power(m, power, 4242))
    k = (1 << power) - 1
    assert int(w.min()) == 1 and int(w.max()) == k
    cnt = np.bincount(w, minlength=k + 1)[1:]
    assert cnt.shape[0] == k and (cnt > 0).all()
    if power == 1:
        assert cnt[0] == m
    else:
        inner = m / (k - 1)
        assert abs(cnt[0] - inner / 2) < 0.1 * inner and abs(cnt[-1] - inner / 2) < 0.1 * inner
        if k > 2:
            assert np.all(np.abs(cnt[1:-1] - inner) < 0.1 * inner + 5 * np.sqrt(inner))


def test_power_variant_keeps_the_topology():
    a = graphgen.workload("rmat12")
    b = graphgen.workload("rmat12p3")
    assert np.array_equal(a.edges.src, b.edges.src) and np.array_equal(a.edges.dst, b.edges.dst)
    assert set(np.unique(b.edges.w).tolist()) <= set(range(1, 8))


def test_workload_weight_kinds_and_labels():
    """binary32_weights / weight_label agree with the weights each named
    workload actually carries."""
    import numpy as np
    cases = {"rmat12": (False, "U{1..255}"), "rmat12f": (True, "binary32, uniform on (0, 1]"),
             "rmat12c5": (True, "binary32, converge(x, 0.5) (Eq. 8)"),
             "rmat12p20": (False, "Eq. 7, power 20: 1..1048575"), "grid64": (False, "U{1..1000}"),
             "grid64w1000000": (False, "U{1..1000000}"), "er12": (False, "U{1..255}")}
    for name, (fw, label) in cases.items():
        assert graphgen.binary32_weights(name) == fw, name
        assert graphgen.weight_label(name) == label, name
        w = graphgen.workload(name).csr.w
        if fw:
            v = w.view(np.float32)
            assert np.all(v > 0) and np.all(v <= 1.0), name
        else:
            hi = {"rmat12p20": (1 << 20) - 1, "grid64w1000000": 1000000, "grid64": 1000}.get(name, 255)
            assert w.min() >= 1 and w.max() <= hi, name
