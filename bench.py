#!/usr/bin/env python
"""Benchmark: plain single-source SSSP on an undirected R-MAT graph of scale 24
(edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), uint32 weights uniform on
1..255), one MI355X.

A step is one solve from a seeded source (sources drawn among vertices of
degree >= 1, the paper's trial protocol, Section 4), graph resident in HBM.
GTEPS = (undirected edges with both endpoints reachable) / solve time.
Graph preparation (the paper's preprocess, Section 4.6) is timed apart.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SSSP GTEPS on RMAT-24 (1 GPU); batched queries/s + p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
INF = 0xFFFFFFFF


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def alg_bytes(c: dict) -> int:
    """Bytes the method itself must move for one solve (counted by the engine):
    16 per expansion (frontier id, dist[u], the row bounds), 12 per pushed edge
    (column, weight, dist[v]), 4 per successful decrease, 12 per pull-list
    entry (id, dist, smallest weight), 12 per pulled edge, 8 per queue entry
    (written once, read once)."""
    return (16 * c["expansions"] + 12 * c["push_scanned"] + 4 * c["relax_success"]
            + 12 * c["pull_vertices"] + 12 * c["pull_scanned"] + 8 * c["queue_entries"])


COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_engine_rmat24_counters.md")
ENGINE_SOURCES = [os.path.join(ROOT, "paper_2506_19349_amd", "csrc", f)
                  for f in ("engine.hip", "engine.h")]


def engine_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ENGINE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per engine launch from the committed counter summary: the
    FETCH_SIZE and WRITE_SIZE readings (KiB per dispatch) of the engine kernel,
    each scaled by what the same counter reads for a copy of known size. None
    when there is no summary for this workload or the engine has changed since."""
    if workload != "rmat24" or not os.path.exists(COUNTERS_FILE):
        return None
    vals = {}
    with open(COUNTERS_FILE) as fh:
        for line in fh:
            m = re.match(r"^\s*-\s*([a-z0-9_]+):\s*([0-9a-f.]+)\s*$", line)
            if m:
                vals[m.group(1)] = m.group(2)
    need = ("engine_source_sha256", "engine_fetch_kib", "engine_write_kib", "copy_bytes",
            "copy_fetch_kib", "copy_write_kib")
    if any(k not in vals for k in need) or vals["engine_source_sha256"] != engine_source_hash():
        return None
    cb = float(vals["copy_bytes"])
    f_fetch = cb / (float(vals["copy_fetch_kib"]) * 1024.0)
    f_write = cb / (float(vals["copy_write_kib"]) * 1024.0)
    return (float(vals["engine_fetch_kib"]) * 1024.0 * f_fetch
            + float(vals["engine_write_kib"]) * 1024.0 * f_write)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with three 1 GiB device-to-device copies (reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs a single-GPU solver "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_2506_19349_amd as sssp

    torch.cuda.set_device(0)
    t = time.time()
    wl = graphgen.workload(args.workload)
    csr = wl.csr
    log("generated %s: n=%d nnz=%d in %.1fs" % (wl.name, csr.n, csr.nnz, time.time() - t))
    deg = csr.degrees()

    torch.cuda.synchronize()
    t = time.perf_counter()
    g = sssp.Graph.from_csr(csr)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t
    info = g.info()
    log("graph prepared on the GPU in %.3fs (highD(0)=%d, max deg %d)"
        % (prep_s, info["high_d0"], info["max_degree"]))

    K, W = args.steps, args.warmup
    sources = [int(s) for s in wl.sources(K + W)]
    outs = [torch.empty(csr.n, dtype=torch.uint32, device="cuda") for _ in range(K)]
    for s in sources[:W]:
        g.solve(s, out=outs[0])
    torch.cuda.synchronize()
    sssp.engine_times()  # discard the warm-up timings

    timed = sources[W:]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, s in enumerate(timed):
        g.solve(s, out=outs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    eng_us = sssp.engine_times()
    total_s = t1 - t0
    log("timed %d solves in %.3f ms" % (K, total_s * 1e3))

    m_cc = []
    for o in outs:
        d = o.cpu().numpy()
        m_cc.append(int(deg[d != INF].sum()) // 2)
    gteps = sum(m_cc) / total_s / 1e9

    # work counters of the same sources (untimed pass; counts vary slightly
    # with relaxation order)
    ctr = []
    for s in timed:
        g.solve(s, out=outs[0])
        ctr.append(sssp.counters())
    sssp.engine_times()
    B = [alg_bytes(c) for c in ctr]
    eng_mean_us = sum(eng_us) / max(len(eng_us), 1)
    achieved = (sum(B) / len(B)) / (eng_mean_us * 1e-6) / 1e9
    n_reach = int((outs[1 if K > 1 else 0].cpu().numpy() != INF).sum())
    c0 = ctr[1 if K > 1 else 0]
    counters = {
        "nTrav": round((c0["push_scanned"] + c0["pull_scanned"]) / max(n_reach, 1), 3),
        "nSync": round((c0["rounds"] + c0["pulls"]) / math.log2(csr.n), 3),
        "steps": c0["steps"], "rounds": c0["rounds"], "ticks": c0["ticks"],
        "relax_success": c0["relax_success"], "expansions": c0["expansions"],
    }
    log("GTEPS %.2f, engine %.1f us/solve, alg bytes %.1f MB/solve -> %.1f GB/s"
        % (gteps, eng_mean_us, sum(B) / len(B) / 1e6, achieved))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import native  # CPU baseline leg only
        log("oracle CPU baseline: building its adjacency from the raw edge list")
        adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
        s = timed[-1]  # outs[0] holds this source's distances from the counters pass
        t = time.perf_counter()
        ref = adj.dijkstra(s)
        dt = time.perf_counter() - t
        adj.close()
        parity = bool(np.array_equal(ref, outs[0].cpu().numpy()))
        cpu = {"value": round(m_cc[-1] / dt / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "binary-heap Dijkstra (the oracle), 1 thread, one source of the same "
                         "RMAT-24 graph, %.1f s; GPU result for it bit-exact: %s" % (dt, parity)}
        log("oracle: %.2f s for one source -> %.4f GTEPS; GPU bit-exact: %s" % (dt, cpu["value"], parity))

    if args.calibrate_copy:
        nb = 1 << 30
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copies done (3 x 1 GiB)")

    traffic = measured_traffic(wl.name)
    config = {"workload": "rmat24-plain-sssp" if wl.name == "rmat24" else wl.name,
              "n": csr.n, "nnz": csr.nnz, "sources": K, "seed": wl.seed,
              "m_cc_mean": int(sum(m_cc) / len(m_cc)), "parallelism": "1 GPU"}
    if wl.name.startswith("rmat"):
        config.update({"edge_factor": 16, "weights": "U{1..255}", "rmat_abc": [0.57, 0.19, 0.19]})
    elif wl.name.startswith("er"):
        config.update({"mean_degree": 32, "weights": "U{1..255}"})
    elif wl.name.startswith("grid"):
        config.update({"edges_kept": 0.95, "diagonals": 0.01, "weights": "U{1..1000}"})
    line = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(total_s * 1e3 / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None if traffic is None else int(traffic),
                     "kernel": "k_engine", "kernel_us_mean": round(eng_mean_us, 2),
                     "alg_bytes_per_launch": int(sum(B) / len(B))},
        "cpu_baseline": cpu,
        "prep_s": round(prep_s, 4),
        "counters": counters,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
