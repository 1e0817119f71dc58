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
# how the oracle used for the CPU baselines was built (set in main)
ORACLE_BUILD = "gcc -O3"


T_START = time.time()


def log(*a):
    print("[bench]", "%6.1fs" % (time.time() - T_START), *a, file=sys.stderr, flush=True)


def alg_bytes(c: dict) -> int:
    """Bytes the method itself must move for one solve (counted by the engine):
    16 per expansion (frontier id, dist[u], the row bounds), 12 per pushed edge
    (column, weight, dist[v]), 4 per successful decrease, 16 per vertex the
    pull examines (an unsettled vertex of degree >= 1: id, dist, row bounds and
    first weight), 12 per pulled edge, 8 per queue entry (written once, read
    once)."""
    return (16 * c["expansions"] + 12 * c["push_scanned"] + 4 * c["relax_success"]
            + 16 * c["pull_unsettled"] + 12 * c["pull_scanned"] + 8 * c["queue_entries"])


def alg_accesses(c: dict) -> int:
    """Random accesses the method itself makes in one solve (counted by the
    engine): one per expansion (the vertex's record), per pushed edge
    (dist[v]), per successful decrease (the atomic), per vertex the pull
    examines and per pulled edge; queue entries are read and written in order
    and are not counted."""
    return (c["expansions"] + c["push_scanned"] + c["relax_success"] + c["pull_unsettled"]
            + c["pull_scanned"])


COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_engine_rmat24_counters.md")
ENGINE_SOURCES = [os.path.join(ROOT, "paper_2506_19349_amd", "csrc", f)
                  for f in ("engine.hip", "engine.h")]


def host_info(torch) -> dict:
    """The machine the numbers come from: host CPU model and thread count (the
    oracle's baselines run there) and the GPU's name."""
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": cpu, "nproc": os.cpu_count(),
            "gpu": torch.cuda.get_device_name(0) if torch.cuda.is_available() else ""}


def engine_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ENGINE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per engine launch from the committed counter summary, or None
    when there is no summary for this workload or the engine has changed since.

    Returns (traffic, copy_scaled, unscaled). traffic: the engine kernel's
    FETCH_SIZE reading (KiB per dispatch) scaled by what the same counter reads
    for a reference gather of known bytes (random 64-byte rows, the engine's own
    access pattern), plus its WRITE_SIZE reading scaled by a copy of known
    size. copy_scaled: both counters scaled by the copy (a streaming read);
    unscaled: the two readings as they stand."""
    if workload != "rmat24" or not os.path.exists(COUNTERS_FILE):
        return None
    vals = {}
    with open(COUNTERS_FILE) as fh:
        for line in fh:
            m = re.match(r"^\s*-\s*([a-z0-9_]+):\s*([0-9a-f.]+)\s*$", line)
            if m:
                vals[m.group(1)] = m.group(2)
    need = ("engine_source_sha256", "engine_fetch_kib", "engine_write_kib", "copy_bytes",
            "copy_fetch_kib", "copy_write_kib", "gather_read_bytes", "gather_fetch_kib")
    if any(k not in vals for k in need) or vals["engine_source_sha256"] != engine_source_hash():
        return None
    fetch = float(vals["engine_fetch_kib"]) * 1024.0
    write = float(vals["engine_write_kib"]) * 1024.0
    cb = float(vals["copy_bytes"])
    f_copy = cb / (float(vals["copy_fetch_kib"]) * 1024.0)
    f_write = cb / (float(vals["copy_write_kib"]) * 1024.0)
    f_gather = float(vals["gather_read_bytes"]) / (float(vals["gather_fetch_kib"]) * 1024.0)
    return fetch * f_gather + write * f_write, fetch * f_copy + write * f_write, fetch + write


def time_solves(sssp, torch, g, srcs, outs, warm, **opts):
    """Solve each source once (outs[i] for srcs[i]) after solving warm[] untimed;
    returns (wall seconds, engine microseconds per solve)."""
    for s in warm:
        g.solve(s, out=outs[0], **opts)
    torch.cuda.synchronize()
    sssp.engine_times()
    t0 = time.perf_counter()
    for i, s in enumerate(srcs):
        g.solve(s, out=outs[i], **opts)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, sssp.engine_times()


def config_section(args, sssp, torch, np, graphgen, name, nsrc, repeat, what):
    """One plain configuration: GTEPS over its seeded sources (each solved
    `repeat` times, after one untimed solve), the engine kernel's mean time
    (HIP events), algorithmic bytes and their fraction of the HBM peak, every
    source's distances against the oracle's Dijkstra (bit for bit), and the
    oracle itself timed on one source, one thread."""
    from oracle import native  # parity and the CPU baseline leg
    t = time.time()
    wl = graphgen.workload(name)
    c = wl.csr
    deg = c.degrees()
    g = sssp.Graph.from_csr(c)
    log("%s: n=%d nnz=%d generated and prepared in %.1fs" % (name, c.n, c.nnz, time.time() - t))
    base = [int(s) for s in wl.sources(nsrc)]
    srcs = [s for s in base for _ in range(repeat)]
    outs = [torch.empty(c.n, dtype=torch.uint32, device="cuda") for _ in base]
    wall, eng = 0.0, []
    for r in range(repeat):
        dt, e = time_solves(sssp, torch, g, base, outs, base[:1] if r == 0 else [])
        wall += dt
        eng += e
    dists = [o.cpu().numpy() for o in outs]
    m_cc = [int(deg[d != INF].sum()) // 2 for d in dists]
    gteps = sum(m_cc) * repeat / wall / 1e9
    ctr = []
    for s in base:
        g.solve(s, out=outs[0])
        ctr.append(sssp.counters())
    sssp.engine_times()
    B = sum(alg_bytes(x) for x in ctr) / len(ctr)
    eng_mean = sum(eng) / max(len(eng), 1)
    del outs
    g.close()
    adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
    threads = max(1, min(16, os.cpu_count() or 1))
    refs = adj.dijkstra_many(base, threads)
    exact = [bool(np.array_equal(refs[i], dists[i])) for i in range(len(base))]
    rec = {"workload": what, "n": c.n, "nnz": c.nnz, "seed": wl.seed, "sources": len(base),
           "solves_timed": len(srcs), "gteps": round(gteps, 4), "ms_per_solve": round(wall * 1e3 / len(srcs), 4),
           "engine_us_mean": round(eng_mean, 2), "alg_bytes_per_solve": int(B),
           "roofline_frac_alg": round(B / (eng_mean * 1e-6) / 1e9 / HBM_PEAK_GBS, 6),
           "parity_vs_oracle": {"sources_checked": len(base), "bit_exact": all(exact)},
           "counters": {"steps": ctr[0]["steps"], "rounds": ctr[0]["rounds"], "ticks": ctr[0]["ticks"],
                        "fused_rounds": ctr[0]["fused_rounds"],
                        "nTrav": round((ctr[0]["push_scanned"] + ctr[0]["pull_scanned"])
                                       / max(int((dists[0] != INF).sum()), 1), 3)}}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        adj.dijkstra(base[0])
        dtc = time.perf_counter() - t0
        rec["cpu_baseline"] = {
            "value": round(m_cc[0] / dtc / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "binary-heap Dijkstra (the oracle, %s), 1 thread, source %d of the same graph, %.2f s"
                      % (ORACLE_BUILD, base[0], dtc)}
    adj.close()
    log("%s: %.3f GTEPS, %.3f ms/solve, engine %.1f us, %d steps, %d ticks; bit-exact on %d sources: %s"
        % (name, gteps, rec["ms_per_solve"], eng_mean, ctr[0]["steps"], ctr[0]["ticks"], len(base), all(exact)))
    return rec


# the autotuner's coordinate-descent search space (sssp_autotune), knob by knob
TUNER_SPACE = {"tile_shape": [1, 2, 3, 4], "blocks_per_cu": [1, 2, "all the shape allows"],
               "heavy_split": [64, 256, 1024, 4096], "fuse_rounds": ["on (256)", "off"],
               "beta": "0.9 (not tuned here; {0.85, 0.9, 0.95} with tune_beta)"}


def tuner_report(rep, tune_s):
    return {"space": TUNER_SPACE, "evaluations": rep["evaluations"], "seconds": round(tune_s, 2),
            "default_us": round(rep["default_us"], 1), "best_us": round(rep["best_us"], 1),
            "gain": round(rep["default_us"] / rep["best_us"], 4) if rep["best_us"] > 0 else None}


def batched_section(args, sssp, torch, np, graphgen):
    """64 sources on RMAT-22 in one graph-captured persistent launch, and 256
    small R-MAT graphs (scales 10..16) in another; knobs picked by the
    autotuner. Parity by the oracle's invariant checker (complete for w >= 1)."""
    from oracle import native  # invariant checker and CPU baseline only
    res = {}
    wl = graphgen.workload("rmat22")
    c = wl.csr
    g = sssp.Graph.from_csr(c)
    k = 64
    srcs = [int(s) for s in wl.sources(4 * k)]
    t = time.perf_counter()
    tuned, rep = sssp.autotune([g] * k, srcs[:k], batched=True)
    tune_s = time.perf_counter() - t
    outs = [torch.empty(c.n, dtype=torch.uint32, device="cuda") for _ in range(k)]
    plan = sssp.Plan([g] * k, outs, **tuned)
    plan.run(srcs[:k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(1, 4):
        plan.run(srcs[r * k:(r + 1) * k])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    last = srcs[3 * k:4 * k]
    ok = all(sum(native.check_sssp(c.n, c.rowptr, c.col, c.w, last[i], outs[i].cpu().numpy())) == 0
             for i in (0, 21, 42, 63))
    one = torch.empty(c.n, dtype=torch.uint32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in last:
        g.solve(s, out=one)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    res["rmat22_64_sources"] = {
        "queries_per_s": round(k / dt, 1), "ms_per_batch": round(dt * 1e3, 3),
        "one_at_a_time_queries_per_s": round(k / dt1, 1), "speedup": round(dt1 / dt, 2),
        "tuned": tuned, "tuner": tuner_report(rep, tune_s), "checked_rows_exact": bool(ok)}
    log("batched RMAT-22 x64: %.1f q/s (one at a time %.1f q/s), tuned %s" % (k / dt, k / dt1, tuned))
    if not args.no_cpu_baseline:
        threads = max(1, min(16, os.cpu_count() or 1))
        adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
        sample = last[:16]
        t0 = time.perf_counter()
        ref = adj.dijkstra_many(sample, threads)
        dtc = time.perf_counter() - t0
        adj.close()
        ok_c = bool(np.array_equal(ref[0], outs[0].cpu().numpy()))
        res["rmat22_64_sources"]["cpu_baseline"] = {
            "value": round(len(sample) / dtc, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "binary-heap Dijkstra (the oracle, %s), %d sources of the same graph on a %d-thread "
                      "pool, %.1f s; first row equals the GPU's: %s" % (ORACLE_BUILD, len(sample), threads, dtc, ok_c)}
    del outs, plan, one
    g.close()

    batch = graphgen.small_rmat_batch()
    gs = [sssp.Graph.from_csr(w.csr) for w in batch]
    ss = [[int(x) for x in w.sources(4)] for w in batch]
    t = time.perf_counter()
    tuned2, rep2 = sssp.autotune(gs, [s[0] for s in ss], batched=True)
    tune_s2 = time.perf_counter() - t
    outs = [torch.empty(w.csr.n, dtype=torch.uint32, device="cuda") for w in batch]
    plan = sssp.Plan(gs, outs, **tuned2)
    plan.run([s[0] for s in ss])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(1, 4):
        plan.run([s[r] for s in ss])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    ok = all(sum(native.check_sssp(batch[i].csr.n, batch[i].csr.rowptr, batch[i].csr.col, batch[i].csr.w,
                                   ss[i][3], outs[i].cpu().numpy())) == 0 for i in (0, 85, 170, 255))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gg, s, o in zip(gs, ss, outs):
        gg.solve(s[3], out=o)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    res["rmat10to16_256_graphs"] = {
        "queries_per_s": round(len(gs) / dt, 1), "ms_per_batch": round(dt * 1e3, 3),
        "one_at_a_time_queries_per_s": round(len(gs) / dt1, 1), "speedup": round(dt1 / dt, 2),
        "tuned": tuned2, "tuner": tuner_report(rep2, tune_s2), "checked_rows_exact": bool(ok)}
    log("batched 256 small graphs: %.1f q/s (one at a time %.1f q/s), tuner %.1f -> %.1f us" % (
        len(gs) / dt, len(gs) / dt1, rep2["default_us"], rep2["best_us"]))
    plan.close()
    for gg in gs:
        gg.close()
    return res


def variants_section(args, sssp, torch, np, graphgen):
    """The integer-power weight variants (Eq. 7) of RMAT-22: the same topology
    with 2^power - 1 distinct weights. Per power: GTEPS over 4 solves and the
    paper's nTrav (Section 4.4: worst with one weight, about 5 or less with 255
    or more); every source's distances pass the oracle's invariant checker."""
    from oracle import native  # the any-size distance check
    out = {}
    for p in (1, 2, 3, 4, 6, 8, 10):
        wl = graphgen.workload("rmat22p%d" % p)
        csr = wl.csr
        deg = csr.degrees()
        g = sssp.Graph.from_csr(csr)
        srcs = [int(s) for s in wl.sources(5)]
        o = torch.empty(csr.n, dtype=torch.uint32, device="cuda")
        g.solve(srcs[0], out=o)
        torch.cuda.synchronize()
        sssp.engine_times()
        m_cc, dt, ntrav, ok = 0, 0.0, [], True
        for s in srcs[1:]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.solve(s, out=o)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            c = sssp.counters()
            d = o.cpu().numpy()
            reach = d != INF
            m_cc += int(deg[reach].sum()) // 2
            ntrav.append((c["push_scanned"] + c["pull_scanned"]) / max(int(reach.sum()), 1))
            ok = ok and sum(native.check_sssp(csr.n, csr.rowptr, csr.col, csr.w, s, d)) == 0
        eng = sssp.engine_times()
        out["power%d" % p] = {"distinct_weights": (1 << p) - 1, "gteps": round(m_cc / dt / 1e9, 3),
                              "ms_per_solve": round(dt * 1e3 / (len(srcs) - 1), 3),
                              "engine_us_mean": round(sum(eng) / max(len(eng), 1), 1),
                              "nTrav": round(sum(ntrav) / len(ntrav), 3), "steps": c["steps"],
                              "ticks": c["ticks"], "invariants_ok": ok}
        log("variant power %d: %.2f GTEPS, nTrav %.2f, %d steps, invariants %s"
            % (p, out["power%d" % p]["gteps"], out["power%d" % p]["nTrav"], c["steps"], ok))
        del o
        g.close()
    # computeST's candidate set: Section 4.1's ST_NUM grid against the exact
    # window of distinct settled distances, for integer weights the window
    # covers (maxW 255: bins narrower than one unit, the window by default;
    # maxW 65535: 64 units, the grid by default)
    for name in ("rmat22p8", "rmat22p16"):
        wl = graphgen.workload(name)
        csr = wl.csr
        deg = csr.degrees()
        g = sssp.Graph.from_csr(csr)
        srcs = [int(s) for s in wl.sources(5)]
        o = torch.empty(csr.n, dtype=torch.uint32, device="cuda")
        rec = {"max_weight": int(csr.w.max()),
               "default": "st_grid" if int(csr.w.max()) > 1024 else "window"}
        sched = {}
        for grid in (False, True):
            g.solve(srcs[0], out=o, st_grid=grid)
            torch.cuda.synchronize()
            sched[grid] = [(x["lb"], x["ub"], x["st"]) for x in sssp.schedule()]
            sssp.engine_times()
            m_cc, dt, ntrav = 0, 0.0, []
            for s in srcs[1:]:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.solve(s, out=o, st_grid=grid)
                torch.cuda.synchronize()
                dt += time.perf_counter() - t0
                c = sssp.counters()
                reach = o.cpu().numpy() != INF
                m_cc += int(deg[reach].sum()) // 2
                ntrav.append((c["push_scanned"] + c["pull_scanned"]) / max(int(reach.sum()), 1))
            eng = sssp.engine_times()
            d = o.cpu().numpy()
            rec["st_grid" if grid else "window"] = {
                "gteps": round(m_cc / dt / 1e9, 3), "engine_us_mean": round(sum(eng) / max(len(eng), 1), 1),
                "nTrav": round(sum(ntrav) / len(ntrav), 3), "steps": c["steps"],
                "invariants_ok": sum(native.check_sssp(csr.n, csr.rowptr, csr.col, csr.w, srcs[-1], d)) == 0}
        rec["same_schedule_first_source"] = sched[False] == sched[True]
        out["computest_" + name] = rec
        log("computeST on %s (maxW %d): window %.2f GTEPS nTrav %.2f | ST_NUM grid %.2f GTEPS nTrav %.2f; "
            "same schedule: %s" % (name, rec["max_weight"], rec["window"]["gteps"], rec["window"]["nTrav"],
                                   rec["st_grid"]["gteps"], rec["st_grid"]["nTrav"], rec["same_schedule_first_source"]))
        del o
        g.close()
    # real weights (binary32): the gr26 graphs' (0, 1] weights and a float-pivot
    # variant (Eq. 8) on the RMAT-22 topology, and the (0, 1] weights on the
    # RMAT-24 topology; 4 solves each with the traversal optimisation (the
    # ST_NUM grid) and 4 without; one source each against the oracle's
    # binary32 Dijkstra
    # Then integer weights beyond the exact selection-threshold window: Eq. 7
    # with power 20 on the RMAT-24 topology (the ST_NUM grid), checked by the
    # oracle's invariant checker.
    for name in ("rmat22f", "rmat22c5", "rmat24f", "rmat24p20"):
        fw = graphgen.binary32_weights(name)
        wl = graphgen.workload(name)
        csr = wl.csr
        deg = csr.degrees()
        g = sssp.Graph.from_csr(csr, float_weights=fw)
        srcs = [int(s) for s in wl.sources(5)]
        o = torch.empty(csr.n, dtype=torch.uint32, device="cuda")
        rec = {"weights": graphgen.weight_label(name)}
        for topt in (True, False):
            g.solve(srcs[0], out=o, traversal_opt=topt)
            torch.cuda.synchronize()
            sssp.engine_times()
            m_cc, dt, ntrav = 0, 0.0, []
            for s in srcs[1:]:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.solve(s, out=o, traversal_opt=topt)
                torch.cuda.synchronize()
                dt += time.perf_counter() - t0
                c = sssp.counters()
                reach = o.cpu().numpy() != INF
                m_cc += int(deg[reach].sum()) // 2
                ntrav.append((c["push_scanned"] + c["pull_scanned"]) / max(int(reach.sum()), 1))
            eng = sssp.engine_times()
            leg = {"gteps": round(m_cc / dt / 1e9, 3), "ms_per_solve": round(dt * 1e3 / (len(srcs) - 1), 3),
                   "engine_us_mean": round(sum(eng) / max(len(eng), 1), 1),
                   "nTrav": round(sum(ntrav) / len(ntrav), 3), "steps": c["steps"], "ticks": c["ticks"]}
            if topt:
                rec.update(leg)
            else:
                rec["filter_off"] = leg
        g.solve(srcs[-1], out=o)
        d = o.cpu().numpy()
        if fw:
            adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
            rec["bit_exact_vs_oracle"] = bool(np.array_equal(adj.dijkstra_f32(srcs[-1]), d))
            adj.close()
            ok = rec["bit_exact_vs_oracle"]
        else:
            rec["invariants_ok"] = sum(native.check_sssp(csr.n, csr.rowptr, csr.col, csr.w, srcs[-1], d)) == 0
            ok = rec["invariants_ok"]
        out[name] = rec
        log("%s %s: %.2f GTEPS, nTrav %.2f (filter off: %.2f GTEPS, nTrav %.2f), %d steps; checked: %s"
            % ("real weights" if fw else "beyond the window", name, rec["gteps"], rec["nTrav"],
               rec["filter_off"]["gteps"], rec["filter_off"]["nTrav"], rec["steps"], ok))
        del o
        g.close()
    return out


def served_section(args, sssp, torch, np, graphgen):
    """Served SSSP over resident graphs (RMAT-20, RMAT-22, RMAT-23 and the
    2048 x 2048 road-like grid): N single-source queries, graph uniform per
    query, sources among each graph's vertices of degree >= 1.

    * Plain FIFO: one solve at a time in arrival order, run for real at the
      arrival rate of the FIFO capacity (lambda = 1.0); its per-query service
      times give FIFO's capacity and its latencies at the other rates (one
      server, one query at a time: finish = max(finish, arrival) + service).
    * Served: the continuous-batching server at saturation (every query
      submitted at once: its capacity), then a Poisson stream at lambda =
      {0.5, 0.8, 1.0, 1.25} x FIFO capacity: throughput, p50 and p99 latency
      from submission to completion. Loads below capacity take the stream's
      first --serve-queries-light queries (a run lasts queries / rate
      seconds); the others all N.
    Every served result is compared with the same query solved alone."""
    names = ["rmat20", "rmat22", "rmat23", "grid2048"]
    wls = [graphgen.workload(nm) for nm in names]
    gs = [sssp.Graph.from_csr(w.csr) for w in wls]
    N = args.serve_queries
    loads = [float(x) for x in args.serve_loads.split(",")]
    rng = np.random.default_rng(graphgen.SEED_BASE + 7)
    which = rng.integers(0, len(gs), size=N)
    unit_gaps = rng.exponential(1.0, size=N)  # a unit-rate Poisson stream, scaled per load
    pools = [[int(x) for x in w.sources(N)] for w in wls]
    queries = [(int(which[q]), pools[int(which[q])][q]) for q in range(N)]
    pct = lambda xs, p: float(np.percentile(np.asarray(xs), p) * 1e3)
    # FIFO capacity, calibrated on 8 queries of each graph
    one = [torch.empty(w.csr.n, dtype=torch.uint32, device="cuda") for w in wls]
    per_graph = []
    for gi, gg in enumerate(gs):
        gg.solve(pools[gi][-1], out=one[gi])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in pools[gi][-9:-1]:
            gg.solve(s, out=one[gi])
        torch.cuda.synchronize()
        per_graph.append((time.perf_counter() - t0) / 8)
    cap0 = 1.0 / (sum(per_graph) / len(per_graph))
    log("served mix: one-at-a-time service %s ms -> FIFO capacity %.2f q/s"
        % ([round(x * 1e3, 2) for x in per_graph], cap0))
    # plain FIFO for real at lambda = 1.0: the solo results are kept for the
    # comparison with the served ones
    arrivals = np.cumsum(unit_gaps) / cap0
    arrivals -= arrivals[0]
    solo = [torch.empty(wls[gi].csr.n, dtype=torch.uint32, device="cuda") for gi, _ in queries]
    service, fifo_lat = [], []
    t_start = time.perf_counter()
    for q, (gi, s) in enumerate(queries):
        now = time.perf_counter() - t_start
        if arrivals[q] > now:
            time.sleep(arrivals[q] - now)
        t0 = time.perf_counter()
        gs[gi].solve(s, out=solo[q])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        service.append(t1 - t0)
        fifo_lat.append(t1 - t_start - arrivals[q])
    fifo_cap = N / sum(service)
    log("plain FIFO at %.2f q/s (run): p50 %.1f ms p99 %.1f ms; capacity over all %d queries %.2f q/s"
        % (cap0, pct(fifo_lat, 50), pct(fifo_lat, 99), N, fifo_cap))

    def fifo_at(rate, nq):
        arr = np.cumsum(unit_gaps[:nq]) / rate
        arr -= arr[0]
        fin, lat = 0.0, []
        for a, sv in zip(arr, service[:nq]):
            fin = max(fin, a) + sv
            lat.append(fin - a)
        return {"queries_per_s": round(nq / fin, 3), "p50_ms": round(pct(lat, 50), 2),
                "p99_ms": round(pct(lat, 99), 2)}

    outs = [torch.empty(wls[gi].csr.n, dtype=torch.uint32, device="cuda") for gi, _ in queries]

    def serve(rate, nq):
        srv = sssp.Server(budget_bytes=args.serve_budget_gib << 30, max_batch=args.serve_slots,
                          ticks_per_launch=args.serve_ticks)
        ids = [srv.add_graph(gg) for gg in gs]
        for o in outs:
            o.fill_(0)
        torch.cuda.synchronize()
        tickets = []
        t0 = time.perf_counter()
        if rate is None:
            arr = np.zeros(nq)
        else:
            arr = np.cumsum(unit_gaps[:nq]) / rate
            arr -= arr[0]
        for q, (gi, s) in enumerate(queries[:nq]):
            delay = arr[q] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(ids[gi], s, outs[q]))
        for t in tickets:
            srv.wait(t)
        infos = [srv.info(t) for t in tickets]
        st = srv.stats()
        srv.close()
        lat = [(i["done_us"] - i["submit_us"]) * 1e-6 for i in infos]
        span = (max(i["done_us"] for i in infos) - min(i["submit_us"] for i in infos)) * 1e-6
        same = all(bool(torch.equal(a, b)) for a, b in zip(outs[:nq], solo[:nq]))
        ok = all(i["status"] == 0 for i in infos)
        return {"queries": nq, "queries_per_s": round(nq / span, 3), "p50_ms": round(pct(lat, 50), 2),
                "p99_ms": round(pct(lat, 99), 2), "peak_in_flight": st["peak_active"],
                "engine_launches": st["launches"], "peak_in_use_bytes": st["peak_in_use_bytes"],
                "all_ok": ok, "equal_to_alone": same}

    sat = serve(None, N)
    log("served at saturation (all %d submitted at once): %.2f q/s; equal to alone: %s"
        % (N, sat["queries_per_s"], sat["equal_to_alone"]))
    sweep = []
    for f in loads:
        rate = f * cap0
        nq = N if f >= 1.0 else min(N, args.serve_queries_light)
        r = serve(rate, nq)
        r.update({"load": f, "arrival_rate_per_s": round(rate, 3)})
        r["plain_fifo"] = fifo_at(rate, nq)
        if f == 1.0:
            r["plain_fifo_run"] = {"queries_per_s": round(N / (t1 - t_start), 3),
                                   "p50_ms": round(pct(fifo_lat, 50), 2), "p99_ms": round(pct(fifo_lat, 99), 2)}
        sweep.append(r)
        log("served at %.2f x FIFO capacity (%.2f q/s), %d queries: %.2f q/s p50 %.1f ms p99 %.1f ms | FIFO "
            "%.2f q/s p50 %.1f p99 %.1f; equal: %s" % (f, rate, nq, r["queries_per_s"], r["p50_ms"], r["p99_ms"],
                                                 r["plain_fifo"]["queries_per_s"], r["plain_fifo"]["p50_ms"],
                                                 r["plain_fifo"]["p99_ms"], r["equal_to_alone"]))
    res = {
        "queries": N, "graphs": names, "slots": args.serve_slots, "ticks_per_launch": args.serve_ticks,
        "budget_bytes": args.serve_budget_gib << 30,
        "one_at_a_time_ms_per_graph": [round(x * 1e3, 3) for x in per_graph],
        "fifo_capacity_per_s": round(cap0, 3), "fifo_capacity_all_queries_per_s": round(fifo_cap, 3),
        "saturation": {"served_queries_per_s": sat["queries_per_s"],
                       "plain_fifo_queries_per_s": round(fifo_cap, 3),
                       "speedup": round(sat["queries_per_s"] / fifo_cap, 2),
                       "equal_to_alone": sat["equal_to_alone"], "all_ok": sat["all_ok"]},
        "sweep": sweep,
        "fifo_note": "plain FIFO was run at load 1.0 over all queries (plain_fifo_run); plain_fifo at each "
                     "load applies one-server FIFO queueing to the service times measured in that run, over "
                     "the same queries as the served run at that load"}
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample of the same stream: the first 8 queries
        # of each graph, each graph's on a thread pool; every result is also
        # compared with what the server returned for that query
        from oracle import native  # CPU baseline leg only
        threads = max(1, min(16, os.cpu_count() or 1))
        per = 8
        picked = {}
        for q, (gi, s) in enumerate(queries):
            lst = picked.setdefault(gi, [])
            if len(lst) < per:
                lst.append(q)
        dtc, nq, agree = 0.0, 0, True
        for gi, qs in sorted(picked.items()):
            w = wls[gi]
            adj = native.Adjacency(w.edges.n, w.edges.src, w.edges.dst, w.edges.w)
            t0c = time.perf_counter()
            ref = adj.dijkstra_many([queries[q][1] for q in qs], threads)
            dtc += time.perf_counter() - t0c
            adj.close()
            nq += len(qs)
            agree = agree and all(np.array_equal(ref[j], outs[q].cpu().numpy()) for j, q in enumerate(qs))
        res["cpu_baseline"] = {
            "value": round(nq / dtc, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "binary-heap Dijkstra (the oracle, %s), the first %d queries of each graph in the "
                      "stream (%d in all), each graph's on a %d-thread pool, %.1f s; all equal the served "
                      "results: %s" % (ORACLE_BUILD, per, nq, threads, dtc, agree)}
        log("served mix on the oracle: %.2f queries/s on %d threads (%d queries, %.1f s); equal: %s"
            % (nq / dtc, threads, nq, dtc, agree))
    del outs, solo, one
    for gg in gs:
        gg.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched measurements")
    ap.add_argument("--no-served", action="store_true", help="skip the served measurements")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the integer-power weight variants of RMAT-22")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other plain configurations (RMAT-14, ER-22, the 2048^2 grid)")
    ap.add_argument("--serve-queries", type=int, default=1024)
    ap.add_argument("--serve-loads", default="0.5,0.8,1.0,1.25",
                    help="arrival rates as fractions of the one-at-a-time (FIFO) capacity of the mix")
    ap.add_argument("--serve-queries-light", type=int, default=256,
                    help="queries of the served runs at loads below FIFO capacity (the stream's first)")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-ticks", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--no-random-rates", action="store_true",
                    help="skip the device's random-access rates (the roofline of roofline.random_access)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with three 1 GiB device-to-device copies (reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--calibrate-gather", action="store_true",
                    help="end with three random gathers of 2^22 distinct 64-byte rows of a 4 GiB "
                         "table (reference kernel of known bytes for random 64-byte reads)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single GPU "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_2506_19349_amd as sssp

    global ORACLE_BUILD
    if not args.no_cpu_baseline:
        # the oracle timed as a CPU baseline is built for the host that runs it
        import tempfile
        from oracle import build as obuild, native
        try:
            native.use_build(obuild.build_for_this_host(tempfile.mkdtemp(prefix="oracle_")))
            ORACLE_BUILD = "gcc -O3 -march=native -ffp-contract=off"
        except Exception as e:  # the portable in-tree build stays in use
            log("oracle: host-tuned build failed (%s); timing the in-tree -O3 build" % e)
            ORACLE_BUILD = "gcc -O3 -ffp-contract=off (in-tree)"
        log("oracle for the CPU baselines: %s" % ORACLE_BUILD)

    torch.cuda.set_device(0)
    t = time.time()
    wl = graphgen.workload(args.workload)
    csr = wl.csr
    log("generated %s: n=%d nnz=%d in %.1fs" % (wl.name, csr.n, csr.nnz, time.time() - t))
    deg = csr.degrees()

    fw = graphgen.binary32_weights(wl.name)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g = sssp.Graph.from_csr(csr, float_weights=fw)
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
    trav = sum(c["push_scanned"] + c["pull_scanned"] for c in ctr) / len(ctr)
    counters = {
        # CSR entries the solves scan (pushed and pulled), per second of the timed run
        "traversed_edges_per_s": round(trav / (total_s / K), 1),
        "nTrav": round((c0["push_scanned"] + c0["pull_scanned"]) / max(n_reach, 1), 3),
        "nSync": round((c0["rounds"] + c0["pulls"]) / math.log2(csr.n), 3),
        "steps": c0["steps"], "rounds": c0["rounds"], "ticks": c0["ticks"],
        "relax_success": c0["relax_success"], "expansions": c0["expansions"],
    }
    log("GTEPS %.2f, engine %.1f us/solve, alg bytes %.1f MB/solve -> %.1f GB/s"
        % (gteps, eng_mean_us, sum(B) / len(B) / 1e6, achieved))

    # the random-access roofline: the method's random accesses per second
    # against the rate the device serves independent random 8-byte reads
    # (measured here, sssp_device_random_rates)
    random_access = None
    if not args.no_random_rates:
        rates = sssp.device_random_rates()
        A = sum(alg_accesses(c) for c in ctr) / len(ctr)
        a_rate = A / (eng_mean_us * 1e-6)
        peak = rates["words8_small_per_s"]
        random_access = {
            "achieved": round(a_rate / 1e9, 3), "peak": round(peak / 1e9, 3), "unit": "G accesses/s",
            "frac": round(a_rate / peak, 4), "accesses_per_launch": int(A),
            "peak_kind": "8-byte words read at random from a 128 MiB array (the per-vertex state's size)",
            "device_rates_g_per_s": {k: round(v / 1e9, 3) for k, v in rates.items() if k.endswith("_per_s")}}
        log("random accesses: %.1f M/solve -> %.2f G/s, %.3f of the device's %.2f G/s random 8-byte reads"
            % (A / 1e6, a_rate / 1e9, a_rate / peak, peak / 1e9))

    # ablation: the traversal-optimisation filter off (st = lb in every step;
    # same distances, more edges traversed)
    ab_src = timed[:4]
    ab_out = torch.empty(csr.n, dtype=torch.uint32, device="cuda")
    g.solve(ab_src[0], out=ab_out, traversal_opt=False)
    torch.cuda.synchronize()
    t0a = time.perf_counter()
    for s in ab_src:
        g.solve(s, out=ab_out, traversal_opt=False)
    torch.cuda.synchronize()
    dt_off = (time.perf_counter() - t0a) / len(ab_src)
    c_off = sssp.counters()
    n_reach_off = int((ab_out.cpu().numpy() != INF).sum())
    del ab_out
    ablation = {"traversal_opt": False, "gteps": round(sum(m_cc[:len(ab_src)]) / len(ab_src) / dt_off / 1e9, 3),
                "ms_per_step": round(dt_off * 1e3, 4),
                "nTrav": round((c_off["push_scanned"] + c_off["pull_scanned"]) / max(n_reach_off, 1), 3)}
    sssp.engine_times()
    log("filter off: %.2f GTEPS, nTrav %.2f" % (ablation["gteps"], ablation["nTrav"]))

    # point-to-point queries: the solve stops once the target is settled;
    # targets drawn among the vertices the first timed source reaches
    d_all = outs[0].cpu().numpy()  # distances of timed[-1] (counters pass)
    reach = np.nonzero(d_all != INF)[0]
    rng = np.random.default_rng(wl.seed + 31)
    pairs = [(timed[i % len(timed)], int(rng.choice(reach))) for i in range(8)]
    p2p_out = torch.empty(csr.n, dtype=torch.uint32, device="cuda")
    g.solve_p2p(pairs[0][0], pairs[0][1], out=p2p_out)
    sssp.engine_times()
    steps_p2p = []
    for s, t in pairs:
        g.solve_p2p(s, t, out=p2p_out)
        steps_p2p.append(sssp.counters()["steps"])
    p2p_us = sssp.engine_times()
    # the last pair's target distance against the full solve of its source
    # (its own buffer: outs[0] still holds timed[-1]'s distances)
    chk = torch.empty(csr.n, dtype=torch.uint32, device="cuda")
    g.solve(pairs[-1][0], out=chk)
    sssp.engine_times()
    exact = int(p2p_out[pairs[-1][1]].item()) == int(chk[pairs[-1][1]].item())
    del p2p_out, chk
    p2p = {"pairs": len(pairs), "engine_us_mean": round(sum(p2p_us) / len(p2p_us), 1),
           "vs_full_solve": round(sum(p2p_us) / len(p2p_us) / eng_mean_us, 3),
           "steps_mean": round(sum(steps_p2p) / len(steps_p2p), 2), "last_target_exact": exact}
    log("point-to-point: %.1f us per query (%.2f of a full solve), %.1f steps; exact: %s"
        % (p2p["engine_us_mean"], p2p["vs_full_solve"], p2p["steps_mean"], exact))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import native  # CPU baseline leg only
        log("oracle CPU baseline: building its adjacency from the raw edge list")
        adj = native.Adjacency(wl.edges.n, wl.edges.src, wl.edges.dst, wl.edges.w)
        s = timed[-1]  # outs[0] holds this source's distances from the counters pass
        t = time.perf_counter()
        ref = adj.dijkstra_f32(s) if fw else adj.dijkstra(s)
        dt = time.perf_counter() - t
        adj.close()
        parity = bool(np.array_equal(ref, outs[0].cpu().numpy()))
        cpu = {"value": round(m_cc[-1] / dt / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "binary-heap Dijkstra (the oracle%s, %s), 1 thread, one source of the same "
                         "%s graph, %.1f s; GPU result for it bit-exact: %s"
                         % (", binary32" if fw else "", ORACLE_BUILD, wl.name, dt, parity)}
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
    if args.calibrate_gather:
        # 2^22 distinct rows of 64 bytes (8 int64) at random positions of a
        # 2^26-row table (4 GiB, beyond the last-level cache): 256 MiB read by
        # 64-byte random gathers, 256 MiB written contiguously
        rows = 1 << 26
        tab = torch.empty((rows, 8), dtype=torch.int64, device="cuda")
        tab.fill_(1)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(wl.seed)
        idx = torch.randperm(rows, device="cuda", generator=gen)[: 1 << 22].contiguous()
        torch.cuda.synchronize()
        for _ in range(3):
            out = torch.index_select(tab, 0, idx)
        torch.cuda.synchronize()
        del tab, idx, out
        log("calibration gathers done (3 x 2^22 random 64-byte rows)")

    batched = None
    served = None
    variants = None
    configs = None
    if wl.name == "rmat24":
        del outs
        g.close()
        if not args.no_configs:
            configs = {
                "rmat14": config_section(args, sssp, torch, np, graphgen, "rmat14", 1, 16,
                                         "R-MAT scale 14, edge factor 16, one seeded source (solved 16 times)"),
                "er22": config_section(args, sssp, torch, np, graphgen, "er22", 8, 2,
                                       "G(n, m), n = 2^22, mean degree 32, 8 seeded sources one at a time"),
                "grid2048": config_section(args, sssp, torch, np, graphgen, "grid2048", 4, 1,
                                           "2048 x 2048 grid, 5% of edges dropped, 1% diagonals, "
                                           "w in 1..1000, 4 seeded sources"),
            }
        if not args.no_batched:
            batched = batched_section(args, sssp, torch, np, graphgen)
        if not args.no_served:
            served = served_section(args, sssp, torch, np, graphgen)
        if not args.no_variants:
            variants = variants_section(args, sssp, torch, np, graphgen)

    traffic = measured_traffic(wl.name)
    config = {"workload": "rmat24-plain-sssp" if wl.name == "rmat24" else wl.name,
              "n": csr.n, "nnz": csr.nnz, "sources": K, "seed": wl.seed,
              "m_cc_mean": int(sum(m_cc) / len(m_cc)), "parallelism": "1 GPU"}
    if wl.name.startswith("rmat"):
        config.update({"edge_factor": 16, "weights": graphgen.weight_label(wl.name),
                       "rmat_abc": [0.57, 0.19, 0.19]})
    elif wl.name.startswith("er"):
        config.update({"mean_degree": 32, "weights": graphgen.weight_label(wl.name)})
    elif wl.name.startswith("grid"):
        config.update({"edges_kept": 0.95, "diagonals": 0.01, "weights": graphgen.weight_label(wl.name)})
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
        "dtype": "f32" if fw else "u32",
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None if traffic is None else int(traffic[0]),
                     "traffic_copy_scaled": None if traffic is None else int(traffic[1]),
                     "traffic_unscaled": None if traffic is None else int(traffic[2]),
                     "kernel": "k_engine", "kernel_us_mean": round(eng_mean_us, 2),
                     "alg_bytes_per_launch": int(sum(B) / len(B)),
                     "random_access": random_access},
        "cpu_baseline": cpu,
        "configs": configs,
        "ablation_filter_off": ablation,
        "batched": batched,
        "served": served,
        "point_to_point": p2p,
        "weight_variants": variants,
        "prep_s": round(prep_s, 4),
        "counters": counters,
        "host": host_info(torch),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
