"""MI355X (gfx950) single-source shortest paths after Yu, Wang and Luo,
"A Heuristic Algorithm for Shortest Path Search" (arXiv 2506.19349).

Python face of the C ABI in include/sssp.h: graphs are prepared on the GPU
(`Graph`), solves run as one persistent HIP launch on a torch stream and write
uint32 distances (UINT32_MAX = unreachable) into torch device tensors.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from typing import Iterable, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import SSSPError

INF = 0xFFFFFFFF

__all__ = ["Graph", "solve_multi", "counters", "schedule", "engine_times", "Plan", "autotune",
           "Server", "SSSPError", "INF", "version", "release_workspaces"]


def version() -> str:
    return _lib.sssp_version().decode()


# Library objects still open at interpreter exit, closed by the exit hook in
# dependency order (servers and plans hold graphs) before the library frees its
# own workspaces: nothing of the library is left for the HIP runtime's teardown.
_open_servers = weakref.WeakSet()
_open_plans = weakref.WeakSet()
_open_graphs = weakref.WeakSet()


def release_workspaces() -> None:
    """Free the library's own per-stream workspaces (sssp_release_workspaces);
    graphs, plans and servers stay. Later solves allocate them again."""
    _lib.check(_lib.sssp_release_workspaces())


def device_random_rates(stream=None) -> dict:
    """Random accesses per second the current device serves, by kind
    (sssp_device_random_rates): 64-byte rows from a 4 GiB table, 8-byte words
    from a 128 MiB and from a 4 GiB array, 64-bit atomicMin on the 128 MiB one."""
    r = _lib.RandomRates()
    _lib.check(_lib.sssp_device_random_rates(ctypes.byref(r), _stream_handle(stream)))
    return {f: getattr(r, f) for f, _ in r._fields_ if f != "reserved"}


@atexit.register
def _close_at_exit():
    for group in (_open_servers, _open_plans, _open_graphs):
        for obj in list(group):
            try:
                obj.close()
            except Exception:
                pass
    try:
        _lib.sssp_release_workspaces()
    except Exception:
        pass


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(getattr(stream, "cuda_stream", stream) or 0)


def _ptr(a):
    """Device or host address of a torch tensor or numpy array (kept alive by the caller)."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _as_i32(a):
    if isinstance(a, np.ndarray):
        return np.ascontiguousarray(a, dtype=np.int32)
    torch = _torch()
    return a.to(torch.int32).contiguous()


def _as_u32(a):
    if isinstance(a, np.ndarray):
        return np.ascontiguousarray(a, dtype=np.uint32)
    torch = _torch()
    if a.dtype == torch.uint32:
        return a.contiguous()
    return a.to(torch.int64).to(torch.uint32).contiguous()


def _options(traversal_opt=True, alpha=None, beta=None, host_driven=False, blocks_per_cu=0,
             heavy_split=0, fuse_rounds=0, tile_shape=0, st_grid=None):
    o = _lib.Options()
    o.traversal_opt = 1 if traversal_opt else -1
    o.alpha = int(alpha or 0)
    o.beta = float(beta or 0.0)
    o.host_driven = 1 if host_driven else 0
    o.blocks_per_cu = int(blocks_per_cu)
    o.heavy_split = int(heavy_split)
    o.fuse_rounds = int(fuse_rounds)
    o.tile_shape = int(tile_shape)
    # None: by the weights; True: the ST_NUM grid; False: the exact window
    o.st_grid = 0 if st_grid is None else (1 if st_grid else -1)
    return o


def _check_out(t, count: int, parent: bool = False, what: str = "out"):
    """An output the kernels write: a contiguous cuda tensor on the current
    device of at least `count` entries, uint32 (distances) or int32 (parents)."""
    torch = _torch()
    want = torch.int32 if parent else torch.uint32
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch cuda tensor" % what)
    if t.device.type != "cuda":
        raise ValueError("%s must be a cuda tensor, not on %s" % (what, t.device))
    if t.device.index != torch.cuda.current_device():
        raise ValueError("%s must be on the current cuda device (cuda:%d), not %s"
                         % (what, torch.cuda.current_device(), t.device))
    if t.dtype != want:
        raise ValueError("%s must be %s, not %s" % (what, want, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() < count:
        raise ValueError("%s holds %d entries, %d needed" % (what, t.numel(), count))
    return t


def _empty_dist(n: int, k: Optional[int] = None):
    torch = _torch()
    shape = (n,) if k is None else (k, n)
    return torch.empty(shape, dtype=torch.uint32, device="cuda")


class Graph:
    """A symmetric CSR graph prepared on the current GPU (sssp_graph_create)."""

    def __init__(self, rowptr, colidx, weight, check_symmetry: bool = True, float_weights: bool = False):
        """float_weights: `weight` holds binary32 bit patterns (uint32) or float32
        values; distances are then binary32 bit patterns (view them as float32)."""
        if float_weights and getattr(weight, "dtype", None) is not None and str(weight.dtype).endswith("float32"):
            weight = weight.view(np.uint32) if isinstance(weight, np.ndarray) else weight.view(_torch().int32)
        rp, ci, w = _as_i32(rowptr), _as_i32(colidx), _as_u32(weight)
        n = int(rp.shape[0]) - 1
        flags = (0 if check_symmetry else 1) | (2 if float_weights else 0)
        h = _lib.sssp_graph_create_ex(n, _ptr(rp), _ptr(ci), _ptr(w), flags)
        if not h:
            _lib.check(_lib.sssp_last_error() or -6)
        self._h = h
        self.n = n
        info = self.info()
        self.nnz = info["nnz"]
        _open_graphs.add(self)

    @classmethod
    def from_csr(cls, csr, check_symmetry: bool = True, float_weights: bool = False) -> "Graph":
        return cls(csr.rowptr, csr.col, csr.w, check_symmetry, float_weights)

    def close(self):
        if getattr(self, "_h", None):
            _lib.sssp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        gi = _lib.GraphInfo()
        _lib.check(_lib.sssp_graph_info_get(self._h, ctypes.byref(gi)))
        return {f: getattr(gi, f) for f, _ in gi._fields_ if f != "reserved"}

    def sorted_rows(self):
        col = np.empty(self.nnz, np.int32)
        w = np.empty(self.nnz, np.uint32)
        _lib.check(_lib.sssp_graph_sorted_rows(self._h, col.ctypes.data, w.ctypes.data))
        return col, w

    def rtow(self) -> np.ndarray:
        out = np.empty(4096, np.uint32)
        _lib.check(_lib.sssp_graph_rtow(self._h, out.ctypes.data))
        return out

    def solve(self, source: int, out=None, stream=None, **opts):
        """Distances from `source` as a uint32 cuda tensor of n entries."""
        out = _empty_dist(self.n) if out is None else _check_out(out, self.n)
        o = _options(**opts)
        _lib.check(_lib.sssp_solve_ex(self._h, int(source), _ptr(out), ctypes.byref(o),
                                      _stream_handle(stream)))
        return out

    def solve_tree(self, source: int, out=None, parent=None, stream=None, **opts):
        """Distances and a shortest-path tree from `source`: (dist, parent), a uint32
        and an int32 cuda tensor of n entries; parent[source] = source, -1 where
        unreachable."""
        out = _empty_dist(self.n) if out is None else _check_out(out, self.n)
        if parent is None:
            torch = _torch()
            parent = torch.empty(self.n, dtype=torch.int32, device="cuda")
        else:
            _check_out(parent, self.n, parent=True, what="parent")
        o = _options(**opts)
        _lib.check(_lib.sssp_solve_tree(self._h, int(source), _ptr(out), _ptr(parent), ctypes.byref(o),
                                        _stream_handle(stream)))
        return out, parent

    def solve_p2p(self, source: int, target: int, out=None, stream=None, **opts):
        """Point-to-point query: the solve stops once `target` is settled. Returns
        (distance of target, the uint32 distance tensor): exact for target and
        for every vertex whose distance is not above it, upper bounds elsewhere. Waits
        for the stream."""
        out = _empty_dist(self.n) if out is None else _check_out(out, self.n)
        o = _options(**opts)
        _lib.check(_lib.sssp_solve_p2p(self._h, int(source), int(target), _ptr(out), ctypes.byref(o),
                                       _stream_handle(stream)))
        return int(out[int(target)].item()), out

    def solve_batch(self, sources: Sequence[int], out=None, stream=None):
        """k sources in one launch: a (k, n) uint32 cuda tensor, row i for sources[i]."""
        srcs = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        k = int(srcs.shape[0])
        out = _empty_dist(self.n, k) if out is None else _check_out(out, k * self.n)
        _lib.check(_lib.sssp_solve_batch(self._h, srcs.ctypes.data, k, _ptr(out),
                                         _stream_handle(stream)))
        return out


def _parent_array(parents, k):
    """ctypes array of k int32 output pointers (None entries stay NULL)."""
    return (ctypes.c_void_p * k)(*[(_ptr(p) if p is not None else None) for p in parents])


def solve_multi(graphs: Sequence[Graph], sources: Sequence[int], outs=None, stream=None,
                targets: Optional[Sequence[int]] = None, trees: bool = False, **opts):
    """Independent (graph, source) pairs in one launch; returns the list of
    distance tensors. targets: None, or one per pair (-1: full solve, else a
    point-to-point query that stops once that vertex is settled). trees: also
    return a shortest-path tree per pair, as (outs, parents)."""
    k = len(graphs)
    if outs is None:
        outs = [_empty_dist(g.n) for g in graphs]
    if len(outs) != k:
        raise ValueError("need %d outputs" % k)
    for g, o in zip(graphs, outs):
        _check_out(o, g.n)
    hs = (ctypes.c_void_p * k)(*[g._h for g in graphs])
    srcs = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    ptrs = (ctypes.c_void_p * k)(*[_ptr(o) for o in outs])
    o = _options(**opts)
    if targets is None and not trees:
        _lib.check(_lib.sssp_solve_multi(ctypes.cast(hs, ctypes.c_void_p), srcs.ctypes.data, k,
                                         ctypes.cast(ptrs, ctypes.c_void_p), ctypes.byref(o),
                                         _stream_handle(stream)))
        return outs
    tg = None if targets is None else np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    parents = None
    par = None
    if trees:
        torch = _torch()
        parents = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in graphs]
        par = _parent_array(parents, k)
    _lib.check(_lib.sssp_solve_multi_ex(ctypes.cast(hs, ctypes.c_void_p), srcs.ctypes.data,
                                        None if tg is None else tg.ctypes.data, k,
                                        ctypes.cast(ptrs, ctypes.c_void_p),
                                        None if par is None else ctypes.cast(par, ctypes.c_void_p),
                                        ctypes.byref(o), _stream_handle(stream)))
    return (outs, parents) if trees else outs


def _counters_dict(c) -> dict:
    return {f: int(getattr(c, f)) for f, _ in c._fields_ if f != "reserved"}


class Plan:
    """A k-instance solve captured once as a HIP graph (sssp_plan_create) and
    replayed with new sources: k sources on one graph, or one source on each
    of k graphs. `outs` are the device tensors every run writes."""

    def __init__(self, graphs: Sequence[Graph], outs, stream=None, parents=None, **opts):
        self.k = len(graphs)
        self.graphs = list(graphs)
        self.outs = list(outs)
        self.parents = None if parents is None else list(parents)
        if len(self.outs) != self.k or (self.parents is not None and len(self.parents) != self.k):
            raise ValueError("need %d outputs" % self.k)
        for i, g in enumerate(self.graphs):
            _check_out(self.outs[i], g.n)
            if self.parents is not None and self.parents[i] is not None:
                _check_out(self.parents[i], g.n, parent=True, what="parent")
        hs = (ctypes.c_void_p * self.k)(*[g._h for g in graphs])
        ptrs = (ctypes.c_void_p * self.k)(*[_ptr(o) for o in self.outs])
        o = _options(**opts)
        if self.parents is None:
            h = _lib.sssp_plan_create(ctypes.cast(hs, ctypes.c_void_p), self.k,
                                      ctypes.cast(ptrs, ctypes.c_void_p), ctypes.byref(o),
                                      _stream_handle(stream))
        else:
            par = _parent_array(self.parents, self.k)
            h = _lib.sssp_plan_create_ex(ctypes.cast(hs, ctypes.c_void_p), self.k,
                                         ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(par, ctypes.c_void_p),
                                         ctypes.byref(o), _stream_handle(stream))
        if not h:
            _lib.check(_lib.sssp_last_error() or -6)
        self._h = h
        _open_plans.add(self)

    def run(self, sources: Sequence[int], stream=None, targets: Optional[Sequence[int]] = None):
        """Replay for new sources (and, optionally, point-to-point targets,
        -1 for a full solve); returns the distance tensors."""
        srcs = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        if srcs.shape[0] != self.k:
            raise ValueError("need %d sources" % self.k)
        if targets is None:
            _lib.check(_lib.sssp_plan_run(self._h, srcs.ctypes.data, _stream_handle(stream)))
        else:
            tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
            if tg.shape[0] != self.k:
                raise ValueError("need %d targets" % self.k)
            _lib.check(_lib.sssp_plan_run_ex(self._h, srcs.ctypes.data, tg.ctypes.data,
                                             _stream_handle(stream)))
        return self.outs

    def counters(self) -> dict:
        c = _lib.Counters()
        st = _lib.sssp_plan_counters(self._h, ctypes.byref(c))
        d = _counters_dict(c)
        _lib.check(st)
        return d

    def close(self):
        if getattr(self, "_h", None):
            _lib.sssp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(graphs: Sequence[Graph], sources: Sequence[int], batched: bool = False,
             tune_beta: bool = False, stream=None, **opts):
    """Pick the fastest launch knobs for the workload (sssp_autotune).
    Returns (options dict usable as solve(**opts), report dict)."""
    k = len(graphs)
    hs = (ctypes.c_void_p * k)(*[g._h for g in graphs])
    srcs = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    o = _options(**opts)
    rep = _lib.TuneReport()
    _lib.check(_lib.sssp_autotune(ctypes.cast(hs, ctypes.c_void_p), srcs.ctypes.data, k,
                                  1 if batched else 0, 1 if tune_beta else 0, ctypes.byref(o),
                                  ctypes.byref(rep), _stream_handle(stream)))
    tuned = {"traversal_opt": o.traversal_opt >= 0, "alpha": o.alpha, "beta": o.beta,
             "blocks_per_cu": o.blocks_per_cu, "heavy_split": o.heavy_split,
             "fuse_rounds": o.fuse_rounds, "tile_shape": o.tile_shape}
    report = {"default_us": rep.default_us, "best_us": rep.best_us, "evaluations": rep.evaluations}
    return tuned, report


class Server:
    """Continuous-batching query server over resident graphs (sssp_server_*)."""

    def __init__(self, budget_bytes: int, max_batch: int = 0, ticks_per_launch: int = 0,
                 max_pending: int = 0, **opts):
        cfg = _lib.ServerConfig()
        cfg.budget_bytes = int(budget_bytes)
        cfg.max_batch = int(max_batch)
        cfg.ticks_per_launch = int(ticks_per_launch)
        cfg.max_pending = int(max_pending)
        o = _options(**opts)
        h = _lib.sssp_server_create(ctypes.byref(cfg), ctypes.byref(o))
        if not h:
            _lib.check(_lib.sssp_last_error() or -6)
        self._h = h
        _open_servers.add(self)
        self._graphs = []
        # outputs of queries not yet released: the pump writes them
        # asynchronously, so they must outlive the caller's own references
        self._outputs = {}

    def add_graph(self, g: Graph) -> int:
        gid = _lib.sssp_server_add_graph(self._h, g._h)
        if gid < 0:
            _lib.check(gid)
        self._graphs.append(g)
        return gid

    def query_bytes(self, graph_id: int) -> int:
        b = _lib.sssp_server_query_bytes(self._h, int(graph_id))
        if b < 0:
            _lib.check(int(b))
        return int(b)

    def submit(self, graph_id: int, source: int, out, target: int = -1, parent=None) -> int:
        """Queue a query; target >= 0 makes it point-to-point, parent (an int32
        cuda tensor of n entries) asks for its shortest-path tree. The server
        keeps references to out and parent until release() or close()."""
        if 0 <= int(graph_id) < len(self._graphs):  # an unknown id is the library's to reject
            n = self._graphs[int(graph_id)].n
            _check_out(out, n)
            if parent is not None:
                _check_out(parent, n, parent=True, what="parent")
        t = ctypes.c_int64(0)
        if target == -1 and parent is None:
            _lib.check(_lib.sssp_server_submit(self._h, int(graph_id), int(source), _ptr(out),
                                               ctypes.byref(t)))
        else:
            _lib.check(_lib.sssp_server_submit_ex(self._h, int(graph_id), int(source), int(target), _ptr(out),
                                                  None if parent is None else _ptr(parent), ctypes.byref(t)))
        self._outputs[t.value] = (out, parent)
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32(0)
        _lib.check(_lib.sssp_server_poll(self._h, ctypes.c_int64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> None:
        _lib.check(_lib.sssp_server_wait(self._h, ctypes.c_int64(ticket)))

    def info(self, ticket: int) -> dict:
        r = _lib.RequestInfo()
        _lib.check(_lib.sssp_server_request_info(self._h, ctypes.c_int64(ticket), ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in r._fields_}

    def release(self, ticket: int) -> None:
        _lib.check(_lib.sssp_server_release(self._h, ctypes.c_int64(ticket)))
        self._outputs.pop(int(ticket), None)

    def stats(self) -> dict:
        s = _lib.ServerStats()
        _lib.check(_lib.sssp_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.sssp_server_destroy(self._h)  # finishes every submitted query first
            self._h = None
        self._outputs = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def counters(stream=None) -> dict:
    """Work counters of the last solve on `stream` (synchronises it)."""
    c = _lib.Counters()
    st = _lib.sssp_get_counters(_stream_handle(stream), ctypes.byref(c))
    d = {f: int(getattr(c, f)) for f, _ in c._fields_ if f != "reserved"}
    _lib.check(st)
    return d


def engine_times(stream=None, cap: int = 256) -> list:
    """Engine-kernel durations (microseconds) of the solves on `stream` since the last call."""
    buf = (ctypes.c_float * cap)()
    n = ctypes.c_int32(0)
    _lib.check(_lib.sssp_engine_times(_stream_handle(stream), buf, cap, ctypes.byref(n)))
    return [float(buf[i]) for i in range(n.value)]


def debug_tick_log(enable_cap: int, stream=None) -> None:
    """Enable (cap > 0) or disable the engine's per-tick log for later solves."""
    _lib.check(_lib.sssp_debug_tick_log(_stream_handle(stream), int(enable_cap)))


def debug_get_tick_log(stream=None, cap: int = 1 << 16):
    """Per-tick log of the last solve: one dict per tick with times in
    microseconds from the engine start (100 MHz clock): `arrive` (last
    workgroup at the barrier), `release` (next tick released), `first`
    and `last` (earliest batch start, latest batch end), `heur` and
    `heur_end` (the step's heuristic, None if none ran), and `batches`, `kind`
    (tick kind | init round << 8 | pull << 9 | step << 16)."""
    buf = np.empty((cap, 8), np.uint64)
    n = ctypes.c_int32(0)
    t0 = ctypes.c_uint64(0)
    _lib.check(_lib.sssp_debug_get_tick_log(_stream_handle(stream), buf.ctypes.data, cap,
                                            ctypes.byref(n), ctypes.byref(t0)))
    m = min(cap, n.value)
    base = t0.value
    us = lambda x: (int(x) - base) / 100.0
    out = []
    for i in range(m):
        e = buf[i]
        out.append({"arrive": us(e[0]), "batches": int(e[1]), "kind": int(e[2]), "release": us(e[3]),
                    "first": us(e[4]) if int(e[4]) != 0xFFFFFFFFFFFFFFFF else None,
                    "last": us(e[5]) if int(e[5]) else None,
                    "heur": us(e[6]) if int(e[6]) else None, "heur_end": us(e[7]) if int(e[7]) else None})
    return out


def schedule(stream=None, cap: int = 1 << 16) -> list:
    """Per-step schedule of the last single-source solve on `stream`."""
    buf = (_lib.Step * cap)()
    n = ctypes.c_int32(0)
    _lib.check(_lib.sssp_get_schedule(_stream_handle(stream), buf, cap, ctypes.byref(n)))
    out = []
    for i in range(min(cap, n.value)):
        s = buf[i]
        out.append({f: int(getattr(s, f)) for f, _ in s._fields_ if f != "reserved"})
    return out
