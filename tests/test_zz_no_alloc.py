"""sssp_solve_noalloc through the C ABI: the allocation-free solve (solver
buffers in the library's fixed device array) gives sssp_solve's distances, on
two calls in a row, the second on a smaller graph (the array keeps the first
call's contents), and rejects a graph too large for the array before writing
anything."""
import numpy as np
import pytest

import graphgen
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19349_amd as sssp  # noqa: E402
from paper_2506_19349_amd import _lib  # noqa: E402


def test_noalloc_equals_solve_on_two_calls():
    stream = torch.cuda.current_stream().cuda_stream
    for name, nsrc in (("rmat14", 3), ("grid40", 2)):  # the second graph is smaller
        wl = graphgen.workload(name)
        g = sssp.Graph.from_csr(wl.csr)
        for s in wl.sources(nsrc):
            s = int(s)
            want = g.solve(s).cpu().numpy()
            out = torch.full((wl.csr.n,), 7, dtype=torch.uint32, device="cuda")
            rc = _lib.sssp_solve_noalloc(g._h, s, out.data_ptr(), stream)
            assert rc == 0, _lib.sssp_last_error_message()
            torch.cuda.current_stream().synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got, want), (name, s)
            assert np.array_equal(got, native.dijkstra(wl.edges.n, wl.edges.src, wl.edges.dst,
                                                       wl.edges.w, s)), (name, s)
        g.close()


def test_noalloc_rejects_a_graph_beyond_its_array():
    wl = graphgen.workload("rmat20")
    g = sssp.Graph.from_csr(wl.csr)
    out = torch.full((wl.csr.n,), 7, dtype=torch.uint32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = _lib.sssp_solve_noalloc(g._h, int(wl.sources(1)[0]), out.data_ptr(), stream)
    assert rc == -3  # SSSP_E_RANGE
    torch.cuda.current_stream().synchronize()
    assert bool((out == 7).all())
    assert _lib.sssp_solve_noalloc(g._h, wl.csr.n, out.data_ptr(), stream) == -1
    g.close()
