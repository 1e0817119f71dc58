"""The boundary by name: sssp_graph_create, sssp_solve, sssp_solve_batch and
sssp_graph_destroy called directly through ctypes (no _ex forms, no package
wrapper), on the 16,384-vertex R-MAT graph, against the oracle's Dijkstra.
Host CSR arrays go in; distances come out in torch device memory on torch's
current stream."""
import ctypes

import numpy as np
import pytest

import graphgen
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_19349_amd import _lib  # noqa: E402

INF = 0xFFFFFFFF


def test_create_solve_batch_destroy_by_name():
    wl = graphgen.workload("rmat14")
    c = wl.csr
    rp = np.ascontiguousarray(c.rowptr, np.int32)
    ci = np.ascontiguousarray(c.col, np.int32)
    w = np.ascontiguousarray(c.w, np.uint32)
    g = _lib.sssp_graph_create(c.n, rp.ctypes.data, ci.ctypes.data, w.ctypes.data)
    assert g, _lib.sssp_last_error_message()
    # the caller keeps ownership of its arrays: they may be dropped now
    del rp, ci, w
    stream = torch.cuda.current_stream().cuda_stream
    srcs = [int(s) for s in wl.sources(5)]
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    refs = [adj.dijkstra(s) for s in srcs]
    adj.close()
    out = torch.full((c.n,), 7, dtype=torch.uint32, device="cuda")
    for s, ref in zip(srcs, refs):
        assert _lib.sssp_solve(g, s, out.data_ptr(), stream) == 0
        torch.cuda.current_stream().synchronize()
        d = out.cpu().numpy()
        assert d[s] == 0
        assert np.array_equal(d, ref), s
    k = len(srcs)
    batch = torch.full((k, c.n), 7, dtype=torch.uint32, device="cuda")
    hs = np.ascontiguousarray(srcs, np.int32)
    assert _lib.sssp_solve_batch(g, hs.ctypes.data, k, batch.data_ptr(), stream) == 0
    torch.cuda.current_stream().synchronize()
    b = batch.cpu().numpy()
    for i in range(k):
        assert np.array_equal(b[i], refs[i]), i
    # argument errors are reported before anything is enqueued: nothing written
    out.fill_(7)
    assert _lib.sssp_solve(g, c.n, out.data_ptr(), stream) == -1
    assert _lib.sssp_solve(g, -1, out.data_ptr(), stream) == -1
    assert _lib.sssp_solve(g, srcs[0], None, stream) == -1
    assert _lib.sssp_solve_batch(g, hs.ctypes.data, 0, batch.data_ptr(), stream) == -1
    torch.cuda.current_stream().synchronize()
    assert bool((out == 7).all())
    assert _lib.sssp_graph_destroy(g) == 0
    assert _lib.sssp_graph_destroy(None) == 0


def test_create_by_name_rejects_bad_csr():
    # not symmetric: (0, 1, 5) has no (1, 0, 5)
    rp = np.array([0, 1, 1], np.int32)
    ci = np.array([1], np.int32)
    w = np.array([5], np.uint32)
    assert not _lib.sssp_graph_create(2, rp.ctypes.data, ci.ctypes.data, w.ctypes.data)
    assert _lib.sssp_last_error() == -2
    # a column out of range
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([1, 2], np.int32)
    w = np.array([1, 1], np.uint32)
    assert not _lib.sssp_graph_create(2, rp.ctypes.data, ci.ctypes.data, w.ctypes.data)
    assert _lib.sssp_last_error() == -1
    assert not _lib.sssp_graph_create(0, rp.ctypes.data, ci.ctypes.data, w.ctypes.data)
    assert _lib.sssp_last_error() == -1
