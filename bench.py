#!/usr/bin/env python
"""Benchmark of the graph hot path on one MI355X.

Workload (default `rmat24`): R-MAT scale 24 (16,777,216 vertices, 16 generated
edges per vertex, a/b/c/d = 0.57/0.19/0.19/0.05, seed 1, symmetrized, self
loops and duplicates dropped), int32 ids and int64 offsets, int32 weights
uniform in [1, 255] (seed 2).  One step = BFS from 64 seeded roots, SSSP from
the same 64 roots, and 20 PageRank iterations (d = 0.85), all GPU-resident
with the graph already in HBM.

Printed: one JSON line with the aggregate traversal rate of the step in GTEPS
(section 5's TEPS: BFS and SSSP count the out-degrees of reached vertices,
PageRank counts |E| per iteration), per-algorithm GTEPS and algorithmic HBM
GB/s, the roofline entry of the dominant kernel (timed with HIP events on the
launching stream over the timed region), and the oracle timed on the host
cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
os.environ.setdefault("TG_TIMING", "1")  # per-kernel HIP-event timing inside libtg

HBM_PEAK_GBS = 8000.0
INF = 2**31 - 1


def kernel_sources_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1312_3018_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# Sources each timed kernel is built from, plus the tuning cache that sets its
# launch shapes (a traffic figure is only reused while these are unchanged).
KERNEL_FILES = {
    "pr_gather": ["pagerank.hip", "pr_sliced.hip", "pr_rows.hip", "kcommon.h", "../tuning_cache.json"],
    "bfs_step": ["bfs.hip", "frontier.hip", "kcommon.h", "../tuning_cache.json"],
    "sssp_relax": ["sssp.hip", "kcommon.h", "../tuning_cache.json"],
    "sssp_pull": ["sssp.hip", "frontier.hip", "kcommon.h", "../tuning_cache.json"],
}


def load_traffic(kernel: str, workload: str):
    """Measured HBM bytes per launch from profiles/traffic.json, if taken on
    the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        ent = d.get(workload, {}).get(kernel)
        if ent and ent.get("sources") == kernel_sources_digest(KERNEL_FILES[kernel]):
            return ent.get("bytes_per_launch")
    except Exception:
        return None
    return None


# Rows of profiles/traffic.json: the pass directories (<algo>_fetch,
# <algo>_write, <algo>_hit) their counters come from, the kernels, and how
# they make up one launch of the bench kernel: "sum" (each launch runs all of
# them: their per-launch means add) or "pool" (each launch is one of them:
# the mean over all their launches).
TRAFFIC_ROWS = {
    "sssp_relax": ("sssp", ["k_sssp_relax<true, 1>", "k_sssp_relax<true, 2>"], "pool"),
    "sssp_pull": ("ssspp", ["k_sssp_pull_heavy"], "sum"),
    "pr_gather": ("pr", ["k_pr_rows<true, int, 8>", "k_pr_long<true>", "k_pr_combine", "k_pr_dsum"], "sum"),
    "bfs_step": ("bfs", ["k_bfs_step<int>"], "sum"),
}
# A 1 GiB device-to-device copy (--copy-calibration) reads FETCH_SIZE =
# 524317 KiB and WRITE_SIZE = 1048576 KiB on MI355X.
FETCH_SCALE = round(1073741824 / (524317 * 1024), 4)
WRITE_SCALE = 1.0


def traffic_from(pmc_dir: str, workload: str = "rmat24") -> dict:
    """profiles/traffic.json from rocprofv3 --pmc counter CSVs: per bench
    kernel, the mean bytes per launch of each of its kernels (FETCH_SIZE and
    WRITE_SIZE in KiB, scaled by the copy calibration), summed, with the L2
    hit rate and the digest of the sources and launch shapes measured."""
    import csv
    import re

    def kname(s):
        m = re.search(r"(k_[a-z_0-9]+)(<[^>(]*>)?", s)
        return m.group(1) + (m.group(2) or "") if m else s.split("(")[0]

    def values_by_kernel(tag):
        agg = {}
        with open(os.path.join(pmc_dir, tag, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                agg.setdefault((kname(r["Kernel_Name"]), r["Counter_Name"]), []).append(float(r["Counter_Value"]))
        return agg

    def per_launch(agg, names, counter, how):
        lists = [agg.get((n, counter), []) for n in names]
        if how == "pool":
            vals = [x for lst in lists for x in lst]
            return (sum(vals) / len(vals) if vals else 0.0), len(vals)
        return sum(sum(lst) / len(lst) for lst in lists if lst), (len(lists[0]) if lists else 0)

    out = {}
    for kernel, (algo, names, how) in TRAFFIC_ROWS.items():
        if not os.path.isdir(os.path.join(pmc_dir, f"{algo}_fetch")):
            continue  # no passes taken for this kernel
        fe, wr, hit = (values_by_kernel(f"{algo}_{kind}") for kind in ("fetch", "write", "hit"))
        f, launches = per_launch(fe, names, "FETCH_SIZE", how)
        f *= FETCH_SCALE * 1024
        w = per_launch(wr, names, "WRITE_SIZE", how)[0] * WRITE_SCALE * 1024
        h = per_launch(hit, names, "TCC_HIT_sum", how)[0]
        m = per_launch(hit, names, "TCC_MISS_sum", how)[0]
        out[kernel] = {"bytes_per_launch": round(f + w), "fetch_bytes": round(f), "write_bytes": round(w),
                       "l2_hit_rate": round(h / max(h + m, 1.0), 4),
                       "sources": kernel_sources_digest(KERNEL_FILES[kernel]),
                       "launches_sampled": launches}
    return {workload: out, "calibration": {"fetch_scale": round(FETCH_SCALE, 4), "write_scale": WRITE_SCALE,
                                           "copy_bytes": 1073741824}}


def gather_reference(n, cols, count=1 << 27, reps=3):
    """A reference for the SSSP relaxation's access pattern, measured
    with torch.index_select (not this library's kernels) on an n-element int32
    array (the distance vector): (a) `count` uniformly random indices; (b) the
    graph's own column array as the index stream, i.e. one read of the
    destination's distance per edge in CSR order -- the relaxation's reads
    without its weights, comparisons and atomics."""
    import torch

    def rate(idx):
        out = torch.empty(idx.numel(), dtype=torch.int32, device="cuda")
        torch.index_select(src, 0, idx, out=out)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            torch.index_select(src, 0, idx, out=out)
        b.record()
        torch.cuda.synchronize()
        return idx.numel() / (a.elapsed_time(b) / 1e3 / reps)

    src = torch.zeros(n, dtype=torch.int32, device="cuda")
    uniform = rate(torch.randint(0, n, (count,), dtype=torch.int64, device="cuda"))
    edge = rate(torch.from_numpy(cols).to("cuda"))
    del src
    torch.cuda.empty_cache()
    return {"uniform_gathers_per_s": round(uniform), "edge_order_gathers_per_s": round(edge),
            "array_elems": n, "edges": int(cols.size),
            "how": "torch.index_select over an n-element int32 array: uniformly random int64 indices, "
                   "and the CSR column array (int32) as indices"}


def host_facts() -> dict:
    """The host the oracle runs on: logical CPUs, the ones this process may
    use, CPU model, sockets and memory (from /proc)."""
    facts = {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}
    try:
        txt = open("/proc/cpuinfo").read()
        models = [ln.split(":", 1)[1].strip() for ln in txt.splitlines() if ln.startswith("model name")]
        facts["cpu_model"] = models[0] if models else None
        facts["sockets"] = len({ln.split(":", 1)[1].strip() for ln in txt.splitlines()
                                if ln.startswith("physical id")}) or None
    except OSError:
        pass
    try:
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemTotal"):
                facts["mem_gib"] = round(int(ln.split()[1]) / 2**20, 1)
    except OSError:
        pass
    return facts


def cpu_baseline(g, w, roots, iters, step_units, max_threads=16):
    """The oracle on the host cores over a bounded sample of the same work,
    in two modes: one thread (the jobs one after another) and all usable
    cores (as many independent jobs of each kind as cores, run at once:
    BFS and SSSP per root, one PageRank iteration per job).  Each kind's
    rate (edges per second) is scaled to one step's edge mix."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    deg = np.diff(g.offsets)

    def run(job):
        kind, arg = job
        if kind == "bfs":
            lev = oracle.bfs(g.offsets, g.cols, arg)
            return int(deg[lev != INF].sum())
        if kind == "sssp":
            d = oracle.sssp(g.offsets, g.cols, w, arg)
            return int(deg[d != INF].sum())
        oracle.pagerank(g.offsets, g.cols, 0.85, 1)
        return g.nnz

    def rates(jobs_by_kind, threads):
        out, wall = {}, {}
        for kind, jobs in jobs_by_kind.items():
            t = time.perf_counter()
            if threads == 1:
                edges = sum(run(j) for j in jobs)
            else:
                with cf.ThreadPoolExecutor(max_workers=threads) as ex:
                    edges = sum(ex.map(run, jobs))
            wall[kind] = time.perf_counter() - t
            out[kind] = edges / wall[kind]
        step_s = sum(step_units[k] / out[k] for k in out if step_units.get(k))
        return sum(step_units.values()) / step_s / 1e9, wall

    facts = host_facts()
    cores = max(1, min(facts["usable_cpus"], max_threads))
    one, wall1 = rates({"bfs": [("bfs", int(r)) for r in roots[:4]], "sssp": [("sssp", int(r)) for r in roots[:2]],
                        "pr": [("pr", 1)]}, 1)
    allc, wallc = rates({"bfs": [("bfs", int(r)) for r in roots[:cores]],
                         "sssp": [("sssp", int(r)) for r in roots[:cores]],
                         "pr": [("pr", 1)] * cores}, cores)
    return {
        "value": round(allc, 4),
        "unit": "GTEPS",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"all-cores mode: {cores} BFS roots, {cores} SSSP roots (Dijkstra) and {cores} independent "
                   f"PageRank iterations of the same graph, each kind's jobs run at once on {cores} threads "
                   f"({sum(wallc.values()):.1f} s); rates per kind scaled to one step's edge mix"),
        "one_thread": {"value": round(one, 4), "cores": 1,
                       "sample": f"4 BFS roots, 2 SSSP roots, 1 PageRank iteration, one after another "
                                 f"({sum(wall1.values()):.1f} s)"},
        "host": facts,
    }


def dist_stats(xs) -> dict:
    """Median, p99, mean and its 95% confidence half-width (Student t)."""
    import numpy as np
    from scipy import stats as st

    a = np.asarray(xs, dtype=np.float64)
    n = a.size
    half = float(st.t.ppf(0.975, n - 1) * a.std(ddof=1) / np.sqrt(n)) if n > 1 else None
    return {"n": int(n), "median": round(float(np.median(a)), 4), "p99": round(float(np.percentile(a, 99)), 4),
            "mean": round(float(a.mean()), 4), "ci95": None if half is None else round(half, 4)}


SERVE_GRAPHS = ["rmat18", "rmat19", "rmat20", "rmat21", "rmat22", "rmat23", "uniform20", "uniform22"]


def serve_run(tg, parts, stream_spec, max_slots, pool=256, log=None, keep=()):
    """Offer a Poisson stream of (graph, kind, root, arrival_s) to a server.
    Returns per-query latencies in ms from the scheduled arrival (time spent
    waiting for an output buffer before submission included), the
    wall-clock span, the server statistics and copies of the outputs of the
    queries whose index is in `keep`."""
    import threading

    import torch

    S = tg.Server(max_slots=max_slots)
    gids = [S.add_graph(P) for (_, P) in parts]
    free = [[torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(pool)] for (g, _) in parts]
    cv = threading.Condition()
    inflight = []
    lat = [None] * len(stream_spec)
    kept = {}
    done_flag = [False]

    def collector():
        while True:
            with cv:
                while not inflight and not done_flag[0]:
                    cv.wait()
                if not inflight and done_flag[0]:
                    return
                i, gi, t, buf, queued_ms = inflight.pop(0)
            lat[i] = queued_ms + S.wait(t) / 1e3
            if i in keep:
                kept[i] = buf.clone()
                torch.cuda.synchronize()
            with cv:
                free[gi].append(buf)
                cv.notify_all()

    th = threading.Thread(target=collector)
    th.start()
    t0 = time.perf_counter()
    for i, (gi, kind, root, at) in enumerate(stream_spec):
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        with cv:
            while not free[gi]:
                cv.wait()
            buf = free[gi].pop()
        queued_ms = max(time.perf_counter() - t0 - at, 0.0) * 1e3
        t = S.submit(gids[gi], kind, root, buf)
        with cv:
            inflight.append((i, gi, t, buf, queued_ms))
            cv.notify_all()
        if log and i and i % 4000 == 0:
            log(f"[serve] submitted {i}/{len(stream_spec)}")
    with cv:
        done_flag[0] = True
        cv.notify_all()
    th.join()
    span = time.perf_counter() - t0
    st = S.stats()
    S.close()
    return lat, span, st, kept


def bench_serve(args):
    """Continuous batching (64 slots) against one query per launch chain on
    the same Poisson streams: at 25/50/90% of the mix's capacity with full
    engines and at the offered rate, each stream lasting about
    --serve-seconds.  Sampled outputs of the batched runs are compared with
    the same queries run alone."""
    import numpy as np
    import torch

    import graphgen
    import paper_1312_3018_amd as tg

    log = lambda m: print(m, file=sys.stderr, flush=True)
    parts = []
    for name in SERVE_GRAPHS:
        g = graphgen.workload(name)
        w = graphgen.weights(g, seed=2)
        G = tg.graph_load_csr(g.n, g.offsets, g.cols, w, symmetric=g.symmetric, validate=False)
        parts.append((g, tg.partition_by_degree(G)))
        log(f"[serve] loaded {name}: V={g.n} E={g.nnz}")
    rng = np.random.default_rng(4)
    cand = [np.nonzero(np.diff(g.offsets) > 0)[0] for (g, _) in parts]

    def make_stream(n, rate):
        gaps = rng.exponential(1.0 / rate, n)
        at = np.cumsum(gaps)
        gi = rng.integers(0, len(parts), n)
        kind = rng.integers(0, 2, n)
        roots = [int(cand[k][rng.integers(len(cand[k]))]) for k in gi]
        return [(int(a), int(b), r, float(t)) for a, b, r, t in zip(gi, kind, roots, at)]

    def summarize(lat, span, warm, st):
        l = np.array([x for x in lat[warm:] if x is not None])
        return {"queries": int(l.size), "p50_ms": round(float(np.percentile(l, 50)), 3),
                "p99_ms": round(float(np.percentile(l, 99)), 3), "mean_ms": round(float(l.mean()), 3),
                "queries_per_s": round(len(lat) / span, 1), "max_concurrent": st["max_concurrent"],
                "supersteps": st["supersteps"]}

    capacity = serve_capacity(tg, parts, log)
    cap = capacity["queries_per_s_full_engines"]
    loads = [("25% of capacity", 0.25 * cap), ("50% of capacity", 0.5 * cap), ("90% of capacity", 0.9 * cap),
             (f"offered {args.serve_rate}/s", float(args.serve_rate))]
    rows, checked, mism = [], 0, 0
    for label, rate in loads:
        n = int(min(args.serve_queries, max(400, rate * args.serve_seconds)))
        warm = n // 10
        stream = make_stream(n, rate)
        keep = set(range(warm, n, max((n - warm) // 10, 1)))
        log(f"[serve] {label}: {n} queries at {rate:.0f}/s, continuous batching")
        lat_b, span_b, st_b, kept = serve_run(tg, parts, stream, 64, log=log, keep=keep)
        log(f"[serve] {label}: the same stream, one query per launch chain")
        lat_s, span_s, st_s, _ = serve_run(tg, parts, stream, 1, log=log)
        rows.append({"load": label, "offered_per_s": round(rate, 1), "queries": n, "warm_up_excluded": warm,
                     "continuous_batching": summarize(lat_b, span_b, warm, st_b),
                     "one_per_launch": summarize(lat_s, span_s, warm, st_s)})
        log(f"[serve] {rows[-1]}")
        for i, out in kept.items():
            gi, kind, root, _ = stream[i]
            g, P = parts[gi]
            solo = (tg.bfs(P, [root]) if kind == 0 else tg.sssp(P, [root]))[0]
            mism += int(not torch.equal(out, solo))
            checked += 1
    top = rows[-1]
    out = {"metric": "p50/p99 query latency from arrival and queries/s (continuous batching vs one query per "
                     "launch chain, same streams)",
           "value": top["continuous_batching"]["p99_ms"], "unit": "ms (p99 at the offered rate)",
           "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "serve: 8 resident graphs (" + ", ".join(SERVE_GRAPHS) +
                                  f"), Poisson streams at 25/50/90% of capacity and {args.serve_rate}/s, "
                                  "50% BFS / 50% SSSP, roots uniform among degree >= 1"},
           "loads": rows, "capacity": capacity,
           "batched_outputs_equal_to_solo": f"{checked - mism}/{checked}"}
    print(json.dumps(out), flush=True)


# The server runs SSSP on graphs of at least this many vertices, whose
# largest out-degree is at least this many times the mean, as single
# searches (its defaults sssp_solo_min_vertices and sssp_solo_min_skew).
SERVE_SOLO_MIN_VERTICES = 1 << 22
SERVE_SOLO_MIN_SKEW = 16.0


def serve_solo(g) -> bool:
    """Whether the server's default rule runs this graph's SSSP queries as
    single searches."""
    import numpy as np
    deg = np.diff(np.asarray(g.offsets))
    mean = float(deg.sum()) / max(g.n, 1)
    skew = float(deg.max()) / mean if mean > 0 else 0.0
    return g.n >= SERVE_SOLO_MIN_VERTICES and skew >= SERVE_SOLO_MIN_SKEW


def serve_capacity(tg, parts, log, batch=64):
    """GPU time per query of each (graph, kind) lane when it is full: one
    batch of `batch` queries through the slot engine, the same queries as
    single searches (several in flight, as the server runs SSSP on large
    graphs), and a few queries one at a time, each after a warm-up.  The
    mix's capacity is the inverse of the mean time per query over the lanes,
    each lane taken the way the server serves it (the queries are spread
    evenly over graphs and kinds)."""
    import numpy as np
    import torch

    import graphgen
    lanes, per_query = [], []
    for gi, (g, P) in enumerate(parts):
        roots = graphgen.sample_roots(g, batch, seed=5)
        out = torch.empty((batch, g.n), dtype=torch.int32, device="cuda")
        for kind, batched, solo in (("bfs", tg.bfs_batched, tg.bfs), ("sssp", tg.sssp_batched, tg.sssp)):
            batched(P, roots[:8], out[:8])
            torch.cuda.synchronize()
            t = time.perf_counter()
            batched(P, roots, out)
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t) / batch
            t = time.perf_counter()
            solo(P, roots[:8], out[:8])
            torch.cuda.synchronize()
            ts = (time.perf_counter() - t) / 8
            row = {"graph": SERVE_GRAPHS[gi], "kind": kind, "ms_per_query_batched": round(tb * 1e3, 3),
                   "ms_per_query_solo": round(ts * 1e3, 3)}
            served = tb
            if kind == "sssp" and serve_solo(g):
                t = time.perf_counter()
                solo(P, roots, out)
                torch.cuda.synchronize()
                served = (time.perf_counter() - t) / batch
                row["ms_per_query_single_searches"] = round(served * 1e3, 3)
            row["served_by"] = "single searches" if served is not tb else "slot engine"
            lanes.append(row)
            per_query.append(served)
        del out
    cap = round(1.0 / float(np.mean(per_query)), 1)
    log(f"[serve] capacity of the mix with full engines: {cap} queries/s")
    return {"queries_per_s_full_engines": cap, "batch": batch, "lanes": lanes}


def bench_bc(args):
    """Batched Brandes BC on RMAT-20 (64/256/1024 sources per call) against one
    source at a time, and 32 uneven R-MAT graphs (scales 12-18) as one union."""
    import numpy as np
    import torch

    import graphgen
    import paper_1312_3018_amd as tg

    log = lambda m: print(m, file=sys.stderr, flush=True)
    g = graphgen.rmat(20)
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True, validate=False)
    P = tg.partition_by_degree(G)
    deg = np.diff(g.offsets)
    stream = torch.cuda.current_stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b), r

    def bc_edges(srcs):  # section 5: twice the edges reached from each source
        lev = tg.bfs_batched(P, srcs)
        return 2 * sum(int(deg[(lev[i] != INF).cpu().numpy()].sum()) for i in range(len(srcs)))

    res = {}
    srcs_all = graphgen.sample_roots(g, 1024, seed=3)
    tg.bc_batched(P, srcs_all[:64])  # warm-up
    for B in (64, 256, 1024):
        srcs = srcs_all[:B]
        ms, _ = timed(lambda: tg.bc_batched(P, srcs))
        res[f"batched_{B}"] = {"ms": round(ms, 2), "gteps": round(bc_edges(srcs) / (ms / 1e3) / 1e9, 2)}
        log(f"[bc] batched B={B}: {ms:.1f} ms")
    srcs = srcs_all[:64]
    ms1, _ = timed(lambda: tg.bc(P, srcs))
    res["one_at_a_time_64"] = {"ms": round(ms1, 2), "gteps": round(bc_edges(srcs) / (ms1 / 1e3) / 1e9, 2)}
    res["speedup_64"] = round(ms1 / res["batched_64"]["ms"], 2)
    # 32 graphs of uneven size in one chain: their disjoint union
    offs, cols, base, ebase, srcs_u = [np.zeros(1, dtype=np.int64)], [], 0, 0, []
    for i in range(32):
        gi = graphgen.rmat(12 + (i % 7), seed=100 + i)
        offs.append(gi.offsets[1:] + ebase)
        cols.append(gi.cols + base)
        srcs_u += (graphgen.sample_roots(gi, 64, seed=3) + base).tolist()
        base += gi.n
        ebase += gi.nnz
    U = tg.graph_load_csr(base, np.concatenate(offs), np.concatenate(cols), symmetric=True, validate=False)
    PU = tg.partition_by_degree(U)
    tg.bc_batched(PU, srcs_u[:64])
    msu, _ = timed(lambda: tg.bc_batched(PU, srcs_u))
    res["multi_graph_32"] = {"vertices": base, "edges": ebase, "sources": len(srcs_u), "ms": round(msu, 2)}
    out = {"metric": "BC-TEPS, batched Brandes BC on RMAT-20 vs one source at a time", "value":
           res["batched_1024"]["gteps"], "unit": "GTEPS (BC, x2 rule)", "higher_is_better": True, "n_gpus": 1,
           "data": "synthetic", "dtype": "sigma f64, delta f32",
           "config": {"workload": f"rmat20: V={g.n}, E={g.nnz}; plus 32 R-MAT graphs of scales 12-18 as one union"},
           "results": res}
    print(json.dumps(out), flush=True)


def bench_cc(args):
    """Connected components (minimum-label propagation) on the bench graph:
    TEPS as section 5 counts them (every directed edge of the symmetrized
    graph once per run)."""
    import torch

    import graphgen
    import paper_1312_3018_amd as tg

    log = lambda m: print(m, file=sys.stderr, flush=True)
    g = graphgen.workload(args.workload_graph)
    log(f"[cc] generated {args.workload_graph}: V={g.n} E={g.nnz}")
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, symmetric=g.symmetric, validate=False)
    P = tg.partition_by_degree(G)
    lab = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for _ in range(max(args.warmup, 1)):
        tg.cc(P, lab)
    torch.cuda.synchronize()
    times = []
    for i in range(args.steps):
        t0 = time.perf_counter()
        tg.cc(P, lab)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        log(f"[cc] run {i + 1}/{args.steps}: {times[-1]:.2f} ms")
    st = tg.tg_last_stats()
    ncomp = int(torch.unique(lab).numel())
    ms = sum(times) / len(times)
    out = {"metric": "GTEPS, connected components (minimum-label propagation)",
           "value": round(g.nnz / (ms / 1e3) / 1e9, 2), "unit": "GTEPS", "higher_is_better": True, "n_gpus": 1,
           "data": "synthetic", "dtype": "int32 labels",
           "config": {"workload": f"{args.workload_graph}: V={g.n}, E={g.nnz}"},
           "ms_per_run": round(ms, 3), "supersteps": st.get("supersteps"), "edges_pushed": st.get("edges_pushed"),
           "components": ncomp, "cc_push_ms": st.get("cc_push_ms")}
    print(json.dumps(out), flush=True)


def bench_mapped(args):
    """The bench graph with its edge arrays in mapped host memory (the
    kernels read neighbour ids over the host link, as for graphs larger than
    device memory): BFS from the bench's roots and PageRank iterations,
    beside the same partition with the edges in device memory."""
    import numpy as np
    import torch

    import graphgen
    import paper_1312_3018_amd as tg

    log = lambda m: print(m, file=sys.stderr, flush=True)
    g = graphgen.workload("rmat24")
    roots = graphgen.sample_roots(g, args.roots, seed=3)
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True, validate=False)
    deg = torch.from_numpy(np.diff(g.offsets)).to("cuda")
    res = {}
    for name, tun in (("device", {}), ("mapped", {"mapped_edges": 1})):
        P = tg.partition_by_degree(G, tuning=json.dumps(tun) if tun else None)
        lev = torch.empty((len(roots), g.n), dtype=torch.int32, device="cuda")
        rank = torch.empty(g.n, dtype=torch.float32, device="cuda")
        tg.bfs(P, roots[:2], lev[:2])
        tg.pagerank(P, 0.85, 1, "uniform", rank)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tg.bfs(P, roots, lev)
        torch.cuda.synchronize()
        t_bfs = time.perf_counter() - t0
        t0 = time.perf_counter()
        tg.pagerank(P, 0.85, args.pr_iters, "uniform", rank)
        torch.cuda.synchronize()
        t_pr = time.perf_counter() - t0
        edges = sum(int(deg[lev[i] != INF].sum().item()) for i in range(len(roots)))
        res[name] = {"bfs_gteps": round(edges / t_bfs / 1e9, 2), "bfs_ms_per_root": round(t_bfs * 1e3 / len(roots), 3),
                     "pagerank_gteps": round(g.nnz * args.pr_iters / t_pr / 1e9, 2),
                     "pagerank_ms_per_iter": round(t_pr * 1e3 / args.pr_iters, 3)}
        log(f"[mapped] {name}: {res[name]}")
        del P
        torch.cuda.synchronize()
    out = {"metric": "GTEPS with the edge arrays in mapped host memory (BFS, PageRank)",
           "value": res["mapped"]["bfs_gteps"], "unit": "GTEPS (BFS)", "higher_is_better": True, "n_gpus": 1,
           "data": "synthetic", "dtype": "int32 (bfs), f32 ranks",
           "config": {"workload": f"rmat24: V={g.n}, E={g.nnz}, {len(roots)} BFS roots, {args.pr_iters} PageRank "
                                  "iterations; neighbour ids in pinned host memory mapped into the GPU"},
           "results": res}
    print(json.dumps(out), flush=True)


def bench_hybrid(args):
    """The hybrid split on a directed R-MAT graph: host threads take the
    highest-degree vertices up to a CPU edge share alpha; BFS and PageRank with
    per-superstep boundary exchange over PCIe."""
    import numpy as np
    import torch

    import graphgen
    import paper_1312_3018_amd as tg

    log = lambda m: print(m, file=sys.stderr, flush=True)
    t = time.perf_counter()
    g = graphgen.rmat(args.hybrid_scale, symmetrize=False)
    log(f"[hybrid] generated rmat{args.hybrid_scale} directed: V={g.n} E={g.nnz} in {time.perf_counter() - t:.0f}s")
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, symmetric=False, validate=False)
    roots = graphgen.sample_roots(g, args.hybrid_roots, seed=3)
    deg = np.diff(g.offsets)
    rows = []
    # alpha = 0: the whole graph on the GPU, for reference
    plan = [("high", 0.0)] + [("high", a) for a in args.alphas] + [("low", 0.3), ("rand", 0.3)]
    for strategy, alpha in plan:
        t = time.perf_counter()
        P = tg.partition_by_degree(G, strategy, alpha, seed=5)
        info = P.info()
        log(f"[hybrid] {strategy} alpha={alpha}: partitioned in {time.perf_counter() - t:.0f}s, "
            f"cpu vertices {info.get('cpu_vertices', 0)}, cpu edges {info.get('cpu_edges', 0)}")
        lev = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
        rank = torch.empty(g.n, dtype=torch.float32, device="cuda")
        # untimed warm-up: first-call set-up (PageRank row blocks) stays out of the timings
        tg.bfs(P, [int(roots[0])], lev)
        tg.pagerank(P, 0.85, 1, "uniform", rank)
        torch.cuda.synchronize()
        bfs_ms, st_b, edges = 0.0, [], 0
        for r in roots:
            t0 = time.perf_counter()
            tg.bfs(P, [int(r)], lev)
            bfs_ms += (time.perf_counter() - t0) * 1e3
            st_b.append(tg.tg_last_stats())
            edges += int(deg[(lev[0] != INF).cpu().numpy()].sum())
        t0 = time.perf_counter()
        tg.pagerank(P, 0.85, args.pr_iters, "uniform", rank)
        pr_ms = (time.perf_counter() - t0) * 1e3
        sp = tg.tg_last_stats()
        rows.append({"strategy": strategy, "alpha": alpha, "cpu_vertices": info.get("cpu_vertices", 0),
                     "cpu_edges": info.get("cpu_edges", 0), "boundary_edges": info.get("boundary_edges", 0),
                     "cpu_boundary_edges": info.get("cpu_boundary_edges", 0),
                     "bfs_ms": round(bfs_ms, 2), "bfs_edges": edges,
                     "beta_raw": info.get("beta_raw", 0), "beta_reduced": info.get("beta_reduced", 0),
                     "bfs_gteps": round(edges / (bfs_ms / 1e3) / 1e9, 3),
                     "bfs_gpu_ms": round(sum(s.get("gpu_ms", 0) for s in st_b), 2),
                     "bfs_cpu_ms": round(sum(s.get("cpu_ms", 0) for s in st_b), 2),
                     "bfs_exchange_ms": round(sum(s.get("exchange_ms", 0) for s in st_b), 2),
                     "bfs_exchange_bytes": int(sum(s.get("exchange_bytes", 0) for s in st_b)),
                     "bfs_h2d_bytes": int(sum(s.get("exchange_h2d_bytes", 0) for s in st_b)),
                     "bfs_cpu_edges": int(sum(s.get("cpu_edges", 0) for s in st_b)),
                     "bfs_supersteps": int(sum(s.get("supersteps", 0) for s in st_b)),
                     "pr_ms_per_iter": round(pr_ms / args.pr_iters, 2),
                     "pr_gteps": round(g.nnz * args.pr_iters / (pr_ms / 1e3) / 1e9, 3),
                     "pr_gpu_ms": round(sp.get("gpu_ms", 0), 2), "pr_cpu_ms": round(sp.get("cpu_ms", 0), 2),
                     "pr_exchange_ms": round(sp.get("exchange_ms", 0), 2),
                     "pr_exchange_bytes": int(sp.get("exchange_bytes", 0)),
                     "pr_cpu_edges": int(sp.get("cpu_edges", 0))})
        log(f"[hybrid] {rows[-1]}")
        del P
    out = {"metric": "hybrid split: GTEPS of BFS and PageRank with host-thread partition",
           "value": max(r["bfs_gteps"] for r in rows), "unit": "GTEPS (BFS, best split)", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic",
           "config": {"workload": f"rmat{args.hybrid_scale} directed: V={g.n}, E={g.nnz}; {len(roots)} BFS roots, "
                                  f"{args.pr_iters} PageRank iterations; host threads = OMP_NUM_THREADS"},
           "rows": rows}
    out["model"] = hybrid_model(rows, g.nnz, log)
    print(json.dumps(out), flush=True)


def pearson(x, y):
    import numpy as np
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    if len(x) < 2 or x.std() == 0 or y.std() == 0:
        return None
    return round(float(np.corrcoef(x, y)[0, 1]), 4)


def hybrid_model(rows, num_edges, log):
    """The performance model of section 3 (Equations 1-4) against the measured
    splits.  Inputs, all measured in the same run:
      r_cpu  the host threads' rate (the local edges they processed / their
             compute time) at the split that gives them the most edges
             (HIGH, largest alpha): the stand-in for a host-only run, which
             this engine does not make;
      c      the copy rate over PCIe: bytes over copy time of the largest
             exchange (PageRank's, 4 bytes per message), in messages/s;
      alpha  the share of edges the host processes (its local edges; the
             boundary edges of both sides are reduced on the GPU);
      beta   messages per edge after the reduction of section 3.4 (one per
             distinct remote vertex and direction).
    Predicted speedup over the host alone (Equation 4):
    1 / (beta r_cpu / c + alpha).  Achieved: (edges traversed / r_cpu) over
    the measured hybrid time, the BFS over the same roots and one PageRank
    iteration."""
    pts_rows = [r for r in rows if r["alpha"] > 0 and r.get("bfs_cpu_ms", 0) > 0]
    if not pts_rows:
        return None
    ref = max((r for r in pts_rows if r["strategy"] == "high"), key=lambda r: r["alpha"], default=pts_rows[0])
    rate = lambda r, alg: r[f"{alg}_cpu_edges"] / (r[f"{alg}_cpu_ms"] / 1e3)
    r_cpu = {"bfs": rate(ref, "bfs"), "pagerank": rate(ref, "pr")}
    big = max(pts_rows, key=lambda r: r.get("pr_exchange_bytes", 0))
    c_bytes = big["pr_exchange_bytes"] / (big["pr_exchange_ms"] / 1e3) if big.get("pr_exchange_ms", 0) > 0 else 0.0
    c = c_bytes / 4.0
    if c <= 0:
        return None
    pts = []
    for r in pts_rows:
        a = r["cpu_edges"] / num_edges
        b = r["beta_reduced"]
        pt = {"strategy": r["strategy"], "alpha_set": r["alpha"], "alpha": round(a, 4), "beta": b,
              "r_cpu_bfs": round(rate(r, "bfs")), "r_cpu_pagerank": round(rate(r, "pr"))}
        for alg, e_trav, t_hyb in (("bfs", r["bfs_edges"], r["bfs_ms"] / 1e3),
                                   ("pagerank", num_edges, r["pr_ms_per_iter"] / 1e3)):
            pred = 1.0 / (b * r_cpu[alg] / c + a)
            ach = (e_trav / r_cpu[alg]) / t_hyb
            pt[alg] = {"predicted": round(pred, 3), "achieved": round(ach, 3), "error": round((ach - pred) / pred, 4)}
        pts.append(pt)
    model = {"r_cpu_eps": {k: round(v) for k, v in r_cpu.items()}, "r_cpu_from": f"{ref['strategy']} alpha={ref['alpha']}",
             "c_bytes_per_s": round(c_bytes), "c_msgs_per_s": round(c), "points": pts}
    for alg in ("bfs", "pagerank"):
        high = [p for p in pts if p["strategy"] == "high"]
        model[alg] = {"correlation_high": pearson([p[alg]["predicted"] for p in high], [p[alg]["achieved"] for p in high]),
                      "correlation_all": pearson([p[alg]["predicted"] for p in pts], [p[alg]["achieved"] for p in pts]),
                      "mean_error": round(sum(p[alg]["error"] for p in pts) / len(pts), 4)}
    log(f"[hybrid] model: {model}")
    return model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--pr-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="steps of the second pass that times every kernel launch with HIP events")
    ap.add_argument("--tuning", default="auto",
                    help="JSON tuning object, 'auto' (autotuner cache if present, else built-in) or 'none'")
    ap.add_argument("--autotune", action="store_true", help="run the autotuner (untimed) and update its cache")
    ap.add_argument("--only", choices=["bfs", "sssp", "pagerank"], default=None,
                    help="run one algorithm per step (for profiling); the JSON line then covers only it")
    ap.add_argument("--serve-queries", type=int, default=20000, help="most queries of one serving stream")
    ap.add_argument("--serve-seconds", type=float, default=8.0, help="arrival span of each serving stream")
    ap.add_argument("--hybrid-scale", type=int, default=27)
    ap.add_argument("--hybrid-roots", type=int, default=8)
    ap.add_argument("--alphas", type=float, nargs="*", default=[0.1, 0.2, 0.3, 0.4, 0.5])
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (to scale HBM byte counters)")
    ap.add_argument("--traffic-from", default=None, metavar="DIR",
                    help="only write profiles/traffic.json from the rocprofv3 --pmc passes under DIR")
    args = ap.parse_args()
    if args.traffic_from:
        d = traffic_from(args.traffic_from)
        d["command"] = "python bench.py --traffic-from <pmc dir>; passes as in profiles/rmat24_hbm_traffic.md"
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d))
        return
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 (sharding across "
                                   "GPUs is not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_1312_3018_amd as tg

    tg.require_native()
    torch.cuda.set_device(0)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "bc":
        return bench_bc(args)
    if args.workload == "hybrid":
        return bench_hybrid(args)
    if args.workload == "mapped":
        return bench_mapped(args)
    if args.workload == "cc":
        args.workload_graph = "rmat24"
        return bench_cc(args)
    t = time.perf_counter()
    g = graphgen.workload(args.workload)
    w = graphgen.weights(g, seed=2)
    roots = graphgen.sample_roots(g, args.roots, seed=3)
    gen_s = time.perf_counter() - t
    print(f"[bench] generated {args.workload}: V={g.n} E={g.nnz} in {gen_s:.1f}s", file=sys.stderr, flush=True)
    t = time.perf_counter()
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, w, symmetric=g.symmetric, validate=False)
    P = tg.partition_by_degree(G, tuning=None if args.tuning in ("auto", "none") else args.tuning)
    print(f"[bench] partitioned in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    from paper_1312_3018_amd import autotune
    key = autotune.graph_key(P)
    tuning_used = "built-in"
    if args.autotune:
        # start from the cached shapes; 16 BFS and 8 SSSP roots keep the
        # per-trial noise below the 2% acceptance margin
        res = autotune.tune(P, roots[:16], roots[:8], pr_iters=5, start=autotune.load_cached(key),
                            log=lambda s: print(s, file=sys.stderr, flush=True))
        autotune.save_cached(key, res)
        print(f"[bench] autotuned {key}: {res['initial_ms']} -> {res['final_ms']} in {res['seconds']}s",
              file=sys.stderr, flush=True)
        tuning_used = "autotuned now"
    elif args.tuning == "auto":
        cached = autotune.load_cached(key)
        if cached:
            tg.partition_retune(P, cached)
            tuning_used = "autotuner cache"
    elif args.tuning != "none":
        tuning_used = "given"

    V, E = g.n, g.nnz
    nr = len(roots)
    levels = torch.empty((nr, V), dtype=torch.int32, device="cuda")
    dist = torch.empty((nr, V), dtype=torch.int32, device="cuda")
    rank = torch.empty((V,), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(stats):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        s_bfs = s_sssp = s_pr = {}
        ev[0].record(stream)
        if args.only in (None, "bfs"):
            tg.bfs(P, roots, levels)
            s_bfs = tg.tg_last_stats()
        ev[1].record(stream)
        if args.only in (None, "sssp"):
            tg.sssp(P, roots, dist)
            s_sssp = tg.tg_last_stats()
        ev[2].record(stream)
        if args.only in (None, "pagerank"):
            tg.pagerank(P, 0.85, args.pr_iters, "uniform", rank)
            s_pr = tg.tg_last_stats()
        ev[3].record(stream)
        stats.append((ev, s_bfs, s_sssp, s_pr))

    # timed region: per-kernel timing events off (they add a few
    # microseconds per launch); a second pass with them on gives the
    # kernels' durations for the roofline
    tg.tg_set_timing(False)
    for i in range(args.warmup):
        step([])
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    wall0 = time.perf_counter()
    for i in range(args.steps):
        step(stats)
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    ms_step = total_ms / args.steps

    # kernel durations: HIP events recorded by libtg around each launch on
    # the launching stream, over a separate timed pass of the same steps
    tg.tg_set_timing(True)
    prof = []
    n_prof = max(1, min(args.steps, args.profile_steps))
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for i in range(n_prof):
        step(prof)
    p1.record(stream)
    torch.cuda.synchronize()
    prof_ms_step = p0.elapsed_time(p1) / n_prof
    tg.tg_set_timing(False)
    print(f"[bench] {n_prof} profiled step(s) done", file=sys.stderr, flush=True)

    # traversed edges (section 5): out-degrees of reached vertices
    deg = torch.from_numpy(np.diff(g.offsets)).to("cuda")
    run_bfs = args.only in (None, "bfs")
    run_sssp = args.only in (None, "sssp")
    run_pr = args.only in (None, "pagerank")
    bfs_edges = sum(int(deg[levels[i] != INF].sum().item()) for i in range(nr)) if run_bfs else 0
    sssp_edges = sum(int(deg[dist[i] != INF].sum().item()) for i in range(nr)) if run_sssp else 0
    bfs_verts = int((levels != INF).sum().item()) if run_bfs else 0
    pr_edges = args.pr_iters * E if run_pr else 0
    step_edges = bfs_edges + sssp_edges + pr_edges

    def phase_list(st, k):
        return [x[0][k].elapsed_time(x[0][k + 1]) for x in st]

    t_bfs, t_sssp, t_pr = (max(sum(phase_list(stats, k)) / len(stats), 1e-9) for k in range(3))
    sb, ss, sp = prof[-1][1], prof[-1][2], prof[-1][3]
    # algorithmic bytes (int32 ids, int64 offsets)
    bfs_bytes = 4.125 * bfs_edges + 20.0 * bfs_verts            # whole top-down BFS, all roots
    pr_bytes_iter = 8.0 * E + 16.0 * V                          # one pull iteration
    # per relaxation the edge (packed id|weight word, or id + weight) and
    # the neighbour's distance; per activation offsets, queue, own distance
    pinfo = tg.partition_info(P)
    packed = bool(pinfo.get("packed_edges")) and pinfo["tuning"].get("sssp_packed", 1) == 1
    sssp_bytes = (8.0 if packed else 12.0) * ss.get("relaxations", 0) + 16.0 * ss.get("activations", 0)
    # what the direction-optimizing BFS kernels read: top-down, per edge
    # scanned its id and visited bit, per vertex expanded its offsets and
    # queue entry; bottom-up, per vertex examined two int32 offsets, per
    # in-edge checked its id and frontier bit
    bfs_step_bytes = (4.125 * sb.get("edges_scanned", 0) + 12.0 * sb.get("vertices_expanded", 0) +
                      8.0 * sb.get("bottom_up_vertices_examined", 0) + 4.125 * sb.get("bottom_up_edges_checked", 0))

    def kern(st, name, nbytes, extra=()):
        # summed launch durations, launches, and the busy time (the union of
        # the launches' intervals: launches of concurrent searches overlap)
        ms = st[name + "_ms"] + sum(st[e + "_ms"] for e in extra)
        busy = st.get(name + "_busy_ms", st[name + "_ms"]) + sum(st.get(e + "_busy_ms", st[e + "_ms"]) for e in extra)
        return dict(ms=ms, busy=busy, n=st[name + "_n"], bytes=nbytes)

    kernels = {}
    if "pr_gather_ms" in sp:
        kernels["pr_gather"] = kern(sp, "pr_gather", pr_bytes_iter * sp["pr_gather_n"])
    elif "pr_rows_ms" in sp:
        kernels["pr_gather"] = kern(sp, "pr_rows", pr_bytes_iter * sp["pr_rows_n"])
    elif "pr_slice_gather_ms" in sp:
        # the XCD-split gather: one iteration = class gathers + their combine
        kernels["pr_gather"] = kern(sp, "pr_slice_gather", pr_bytes_iter * sp["pr_slice_gather_n"], ("pr_combine",))
    if "bfs_step_ms" in sb:
        kernels["bfs_step"] = kern(sb, "bfs_step", bfs_step_bytes)
    if "sssp_relax_ms" in ss:
        kernels["sssp_relax"] = kern(ss, "sssp_relax", sssp_bytes)
    if "sssp_pull_ms" in ss:
        # a bucket's heavy edges pulled: per unsettled vertex its offsets,
        # light count and distance, per edge checked its packed word and the
        # member bit of its source
        kernels["sssp_pull"] = kern(ss, "sssp_pull", 4.125 * ss.get("heavy_pull_edges_checked", 0) +
                                    16.0 * ss.get("heavy_pull_vertices", 0))
    roofs = {}
    for k, v in kernels.items():
        n = max(v["n"], 1)
        # a launch's effective duration: busy time over launches (equal to the
        # mean launch duration when launches do not overlap)
        eff_ms = v["busy"] / n
        bytes_per_launch = v["bytes"] / n
        achieved = bytes_per_launch / (eff_ms / 1e3) / 1e9
        tr = load_traffic(k, args.workload)
        # the same bytes over the mean launch duration (which, with launches
        # of concurrent searches overlapping, also counts their waits)
        on_mean = bytes_per_launch / (v["ms"] / n / 1e3) / 1e9 if v["ms"] > 0 else 0.0
        roofs[k] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "frac_on_mean_launch": round(on_mean / HBM_PEAK_GBS, 4),
                    "traffic": tr, "algorithmic_bytes_per_launch": round(bytes_per_launch),
                    "avg_launch_ms": round(v["ms"] / n, 5), "busy_ms_per_launch": round(eff_ms, 5),
                    "launches": int(v["n"]), "share_of_step": round(v["busy"] / prof_ms_step, 4)}
    dominant = max(kernels, key=lambda k: kernels[k]["busy"]) if kernels else None

    # per-root latency: each root alone (one search in flight)
    lat = {}
    if run_bfs:
        one = torch.empty((1, V), dtype=torch.int32, device="cuda")
        xs = []
        for r in roots:
            a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a_.record(stream)
            tg.bfs(P, [int(r)], one)
            b_.record(stream)
            b_.synchronize()
            xs.append(a_.elapsed_time(b_))
        lat["bfs_ms"] = dist_stats(xs)
    if run_sssp:
        one = torch.empty((1, V), dtype=torch.int32, device="cuda")
        xs = []
        for r in roots:
            a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a_.record(stream)
            tg.sssp(P, [int(r)], one)
            b_.record(stream)
            b_.synchronize()
            xs.append(a_.elapsed_time(b_))
        lat["sssp_ms"] = dist_stats(xs)
    print("[bench] single-root latency pass done", file=sys.stderr, flush=True)

    out = {
        "metric": "GTEPS (BFS + SSSP + PageRank step) on RMAT-24",
        "value": round(step_edges / (ms_step / 1e3) / 1e9, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 (bfs/sssp); pagerank: f32 ranks and contributions, per-class partial sums rounded to f32, "
                 "combined in f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: V={V}, E={E} directed (symmetrized), {nr} BFS roots + {nr} "
                               f"SSSP roots (weights 1..255) + {args.pr_iters} PageRank iterations",
                   "global_batch": nr, "parallelism": "none (1 GPU)"},
        "bfs": {"gteps": round(bfs_edges / (t_bfs / 1e3) / 1e9, 2), "ms_per_root": round(t_bfs / nr, 4),
                "hbm_gbs_top_down_equivalent": round(bfs_bytes / (t_bfs / 1e3) / 1e9, 1),
                "hbm_gbs_kernel_bytes": round(bfs_step_bytes / (t_bfs / 1e3) / 1e9, 1),
                "graph500_undirected_gteps": round(bfs_edges / 2 / (t_bfs / 1e3) / 1e9, 2),
                "top_down_edges_per_root": round(sb.get("edges_scanned", 0) / nr),
                "bottom_up_edges_checked_per_root": round(sb.get("bottom_up_edges_checked", 0) / nr),
                "bottom_up_vertices_examined_per_root": round(sb.get("bottom_up_vertices_examined", 0) / nr),
                "bottom_up_steps_per_root": round(sb.get("bottom_up_steps", 0) / nr, 2),
                "supersteps_per_root": round(sb.get("supersteps", 0) / nr, 2),
                "ms_per_root_over_steps": dist_stats([x / nr for x in phase_list(stats, 0)])},
        "sssp": {"gteps": round(sssp_edges / (t_sssp / 1e3) / 1e9, 2), "ms_per_root": round(t_sssp / nr, 4),
                 "supersteps_per_root": round(ss.get("supersteps", 0) / nr, 1),
                 "work_efficiency": round(ss.get("relaxations", 0) / max(sssp_edges, 1), 3),
                 "heavy_pull_edges_checked_per_root": round(ss.get("heavy_pull_edges_checked", 0) / nr),
                 "heavy_pulls_per_root": round(ss.get("pull_supersteps", 0) / nr, 2),
                 "ms_per_root_over_steps": dist_stats([x / nr for x in phase_list(stats, 1)])},
        "gather_reference": None,
        "pagerank": {"gteps": round(pr_edges / (t_pr / 1e3) / 1e9, 2),
                     "ms_per_iter": round(t_pr / args.pr_iters, 4),
                     "hbm_gbs_algorithmic": round(pr_bytes_iter * args.pr_iters / (t_pr / 1e3) / 1e9, 1),
                     "ms_per_iter_over_steps": dist_stats([x / args.pr_iters for x in phase_list(stats, 2)])},
        "single_root_latency": lat,
        "roofline": dict(roofs[dominant], kernel=dominant) if dominant else None,
        "kernels": roofs,
        "profiled_ms_per_step": round(prof_ms_step, 3),
        "tuning": {"source": tuning_used, "values": tg.partition_info(P)["tuning"]},
        "host_wall_s": round(wall, 3),
    }
    if run_sssp and "sssp_relax_ms" in ss:
        gc = gather_reference(V, g.cols)
        relax_rate = ss.get("relaxations", 0) / (ss["sssp_relax_ms"] / 1e3)
        gc["sssp_relaxations_per_s"] = round(relax_rate)
        gc["sssp_relax_vs_edge_order"] = round(relax_rate / gc["edge_order_gathers_per_s"], 3)
        out["gather_reference"] = gc
    if not args.no_cpu_baseline:
        units = {"bfs": bfs_edges, "sssp": sssp_edges, "pr": pr_edges}
        print("[bench] timing the oracle on the host (bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, w, roots, args.pr_iters, units)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
