"""ctypes marshalling for libsssp.so (the C ABI declared in include/sssp.h).

Argument marshalling only: every step of the computation runs in the HIP
library. PyTorch supplies device memory and streams. If the library has not
been built, importing raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsssp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libsssp.so is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
        "(or paper_2506_19349_amd/build.py) first")

# torch's HIP runtime comes up before the library's first HIP call (the
# library works on torch's device memory and streams)
import torch as _torch_rt  # noqa: E402

_torch_rt.cuda.is_available()

lib = ctypes.CDLL(LIB_PATH)

i32 = ctypes.c_int32
u32 = ctypes.c_uint32
vp = ctypes.c_void_p
i32p = ctypes.POINTER(ctypes.c_int32)
u32p = ctypes.POINTER(ctypes.c_uint32)


class Options(ctypes.Structure):
    _fields_ = [("traversal_opt", i32), ("alpha", i32), ("beta", ctypes.c_double),
                ("host_driven", i32), ("blocks_per_cu", i32), ("heavy_split", i32),
                ("fuse_rounds", i32), ("tile_shape", i32), ("st_grid", i32),
                ("reserved", i32 * 6)]


class Counters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "expansions", "band_expansions", "push_scanned", "pull_vertices", "pull_scanned",
        "relax_success", "queue_entries", "rounds", "pulls", "steps", "ticks", "fused_rounds",
        "pull_unsettled")] + [
        ("high_d0", u32), ("gap0", u32), ("flags", u32), ("reserved", u32)]


class Step(ctypes.Structure):
    _fields_ = [("lb", u32), ("ub", u32), ("st", u32), ("rounds", u32), ("pulled", u32),
                ("L", u32), ("S", ctypes.c_uint64), ("h", u32), ("gap", u32), ("st_next", u32),
                ("reserved", u32)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", i32), ("nnz", i32), ("nonisolated", i32), ("max_degree", i32),
                ("distinct_degrees", i32), ("max_weight", u32), ("high_d0", u32),
                ("hub_first", u32), ("device_bytes", ctypes.c_uint64)]


class TuneReport(ctypes.Structure):
    _fields_ = [("default_us", ctypes.c_double), ("best_us", ctypes.c_double),
                ("evaluations", i32), ("reserved", i32 * 7)]


class RandomRates(ctypes.Structure):
    _fields_ = [("rows64_per_s", ctypes.c_double), ("words8_small_per_s", ctypes.c_double),
                ("words8_large_per_s", ctypes.c_double), ("atomics8_small_per_s", ctypes.c_double),
                ("accesses", ctypes.c_int64), ("reserved", i32 * 6)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_batch", i32), ("ticks_per_launch", i32),
                ("max_pending", i32), ("reserved", i32 * 5)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", i32), ("status", i32), ("graph_id", i32), ("source", i32), ("slot", i32),
                ("launches", u32), ("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("done_us", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("engine_us", ctypes.c_double), ("now_us", ctypes.c_double),
                ("budget_bytes", ctypes.c_uint64), ("allocated_bytes", ctypes.c_uint64),
                ("peak_allocated_bytes", ctypes.c_uint64), ("peak_in_use_bytes", ctypes.c_uint64),
                ("active", i32), ("peak_active", i32), ("queued", i32), ("max_batch", i32)]


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


sssp_graph_create = _sig("sssp_graph_create", vp, i32, vp, vp, vp)
sssp_graph_create_ex = _sig("sssp_graph_create_ex", vp, i32, vp, vp, vp, i32)
sssp_graph_destroy = _sig("sssp_graph_destroy", i32, vp)
sssp_graph_info_get = _sig("sssp_graph_info_get", i32, vp, ctypes.POINTER(GraphInfo))
sssp_graph_sorted_rows = _sig("sssp_graph_sorted_rows", i32, vp, vp, vp)
sssp_graph_rtow = _sig("sssp_graph_rtow", i32, vp, vp)
sssp_solve = _sig("sssp_solve", i32, vp, i32, vp, vp)
sssp_solve_ex = _sig("sssp_solve_ex", i32, vp, i32, vp, ctypes.POINTER(Options), vp)
sssp_solve_tree = _sig("sssp_solve_tree", i32, vp, i32, vp, vp, ctypes.POINTER(Options), vp)
sssp_solve_p2p = _sig("sssp_solve_p2p", i32, vp, i32, i32, vp, ctypes.POINTER(Options), vp)
sssp_solve_batch = _sig("sssp_solve_batch", i32, vp, vp, i32, vp, vp)
sssp_solve_multi = _sig("sssp_solve_multi", i32, vp, vp, i32, vp, ctypes.POINTER(Options), vp)
sssp_solve_multi_ex = _sig("sssp_solve_multi_ex", i32, vp, vp, vp, i32, vp, vp, ctypes.POINTER(Options), vp)
sssp_get_counters = _sig("sssp_get_counters", i32, vp, ctypes.POINTER(Counters))
sssp_get_schedule = _sig("sssp_get_schedule", i32, vp, ctypes.POINTER(Step), i32, i32p)
sssp_engine_times = _sig("sssp_engine_times", i32, vp, ctypes.POINTER(ctypes.c_float), i32, i32p)
sssp_debug_tick_log = _sig("sssp_debug_tick_log", i32, vp, i32)
sssp_debug_get_tick_log = _sig("sssp_debug_get_tick_log", i32, vp, vp, i32, i32p,
                               ctypes.POINTER(ctypes.c_uint64))
sssp_plan_create = _sig("sssp_plan_create", vp, vp, i32, vp, ctypes.POINTER(Options), vp)
sssp_plan_run = _sig("sssp_plan_run", i32, vp, vp, vp)
sssp_plan_create_ex = _sig("sssp_plan_create_ex", vp, vp, i32, vp, vp, ctypes.POINTER(Options), vp)
sssp_plan_run_ex = _sig("sssp_plan_run_ex", i32, vp, vp, vp, vp)
sssp_plan_counters = _sig("sssp_plan_counters", i32, vp, ctypes.POINTER(Counters))
sssp_plan_destroy = _sig("sssp_plan_destroy", i32, vp)
sssp_autotune = _sig("sssp_autotune", i32, vp, vp, i32, i32, i32, ctypes.POINTER(Options),
                     ctypes.POINTER(TuneReport), vp)
sssp_server_create = _sig("sssp_server_create", vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(Options))
sssp_server_add_graph = _sig("sssp_server_add_graph", i32, vp, vp)
sssp_server_query_bytes = _sig("sssp_server_query_bytes", ctypes.c_int64, vp, i32)
sssp_server_submit = _sig("sssp_server_submit", i32, vp, i32, i32, vp, ctypes.POINTER(ctypes.c_int64))
sssp_server_submit_ex = _sig("sssp_server_submit_ex", i32, vp, i32, i32, i32, vp, vp,
                             ctypes.POINTER(ctypes.c_int64))
sssp_server_poll = _sig("sssp_server_poll", i32, vp, ctypes.c_int64, i32p)
sssp_server_wait = _sig("sssp_server_wait", i32, vp, ctypes.c_int64)
sssp_server_request_info = _sig("sssp_server_request_info", i32, vp, ctypes.c_int64,
                                ctypes.POINTER(RequestInfo))
sssp_server_release = _sig("sssp_server_release", i32, vp, ctypes.c_int64)
sssp_server_get_stats = _sig("sssp_server_get_stats", i32, vp, ctypes.POINTER(ServerStats))
sssp_server_destroy = _sig("sssp_server_destroy", i32, vp)
sssp_solve_noalloc = _sig("sssp_solve_noalloc", i32, vp, i32, vp, vp)
sssp_release_workspaces = _sig("sssp_release_workspaces", i32)
sssp_device_random_rates = _sig("sssp_device_random_rates", i32, ctypes.POINTER(RandomRates), vp)
sssp_last_error = _sig("sssp_last_error", i32)
sssp_last_error_message = _sig("sssp_last_error_message", ctypes.c_char_p)
sssp_status_str = _sig("sssp_status_str", ctypes.c_char_p, i32)
sssp_version = _sig("sssp_version", ctypes.c_char_p)

STATUS = {0: "SSSP_OK", -1: "SSSP_E_INVAL", -2: "SSSP_E_NOT_SYMMETRIC", -3: "SSSP_E_RANGE",
          -4: "SSSP_E_DIST_OVERFLOW", -5: "SSSP_E_NOMEM", -6: "SSSP_E_DEVICE", -7: "SSSP_E_BUSY"}


class SSSPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, str(status)), message))
        self.status = status


def check(status: int):
    if status != 0:
        raise SSSPError(status, sssp_last_error_message().decode(errors="replace"))
