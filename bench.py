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


# Sources each timed kernel is built from (a traffic figure is only reused
# while these are unchanged).
KERNEL_FILES = {
    "pr_gather": ["pagerank.hip", "kcommon.h"],
    "bfs_expand": ["bfs.hip", "kcommon.h"],
    "sssp_relax": ["sssp.hip", "kcommon.h"],
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


def cpu_baseline(g, w, roots, iters, step_units):
    """The oracle on the host cores over a bounded sample of the same work."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    deg = np.diff(g.offsets)
    jobs = [("bfs", int(r)) for r in roots[:4]] + [("sssp", int(r)) for r in roots[:2]] + [("pr", 1)]

    def run(job):
        kind, arg = job
        t = time.perf_counter()
        if kind == "bfs":
            lev = oracle.bfs(g.offsets, g.cols, arg)
            edges = int(deg[lev != INF].sum())
        elif kind == "sssp":
            d = oracle.sssp(g.offsets, g.cols, w, arg)
            edges = int(deg[d != INF].sum())
        else:
            oracle.pagerank(g.offsets, g.cols, 0.85, arg)
            edges = g.nnz * arg
        return kind, edges, time.perf_counter() - t

    threads = min(len(jobs), os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(run, jobs))
    wall = time.perf_counter() - t0
    per = {}
    for kind, edges, secs in res:
        e, s = per.get(kind, (0, 0.0))
        per[kind] = (e + edges, s + secs)
    # thread-seconds per edge of each kind, scaled to one step's edge mix, then
    # divided by the threads that ran concurrently
    cpu_seconds = sum(step_units[k] * (per[k][1] / per[k][0]) for k in per if per[k][0] > 0)
    step_edges = sum(step_units.values())
    gteps = step_edges / (cpu_seconds / threads) / 1e9
    return {
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{len(roots[:4])} BFS roots, {len(roots[:2])} SSSP roots (Dijkstra) and 1 PageRank "
                   f"iteration of the same graph, run concurrently on {threads} threads in {wall:.1f} s; "
                   "per-kind seconds per edge scaled to one step's edge mix"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--pr-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default="auto",
                    help="JSON tuning object, 'auto' (autotuner cache if present, else built-in) or 'none'")
    ap.add_argument("--autotune", action="store_true", help="run the autotuner (untimed) and update its cache")
    ap.add_argument("--only", choices=["bfs", "sssp", "pagerank"], default=None,
                    help="run one algorithm per step (for profiling); the JSON line then covers only it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (to scale HBM byte counters)")
    args = ap.parse_args()
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
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in DESIGN.md but not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_1312_3018_amd as tg

    tg.require_native()
    torch.cuda.set_device(0)
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
        res = autotune.tune(P, roots[:4], roots[:2], pr_iters=5,
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

    def phase(k):
        return sum(s[0][k].elapsed_time(s[0][k + 1]) for s in stats) / len(stats)

    t_bfs, t_sssp, t_pr = (max(phase(k), 1e-9) for k in range(3))
    last = stats[-1]
    sb, ss, sp = last[1], last[2], last[3]
    # algorithmic bytes (int32 ids, int64 offsets)
    bfs_bytes = 4.125 * bfs_edges + 20.0 * bfs_verts            # whole BFS, all roots
    pr_bytes_iter = 8.0 * E + 16.0 * V                          # one pull iteration
    sssp_bytes = 12.0 * ss.get("relaxations", 0) + 16.0 * ss.get("activations", 0)

    kernels = {}
    if "pr_gather_ms" in sp:
        kernels["pr_gather"] = dict(ms=sp["pr_gather_ms"], n=sp["pr_gather_n"], bytes=pr_bytes_iter * sp["pr_gather_n"])
    if "bfs_expand_ms" in sb:
        exp_bytes = 4.125 * sb["edges_scanned"] + 12.0 * sb["vertices_expanded"]
        kernels["bfs_expand"] = dict(ms=sb["bfs_expand_ms"], n=sb["bfs_expand_n"], bytes=exp_bytes)
    if "sssp_relax_ms" in ss:
        kernels["sssp_relax"] = dict(ms=ss["sssp_relax_ms"], n=ss["sssp_relax_n"], bytes=sssp_bytes)
    roofs = {}
    for k, v in kernels.items():
        avg_ms = v["ms"] / max(v["n"], 1)
        bytes_per_launch = v["bytes"] / max(v["n"], 1)
        achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
        tr = load_traffic(k, args.workload)
        roofs[k] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": tr, "algorithmic_bytes_per_launch": round(bytes_per_launch),
                    "avg_launch_ms": round(avg_ms, 5), "launches": int(v["n"]), "share_of_step":
                        round(v["ms"] / ms_step, 4)}
    dominant = max(kernels, key=lambda k: kernels[k]["ms"]) if kernels else None

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
        "dtype": "int32 (bfs/sssp), f32 ranks with f64 sums (pagerank)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: V={V}, E={E} directed (symmetrized), {nr} BFS roots + {nr} "
                               f"SSSP roots (weights 1..255) + {args.pr_iters} PageRank iterations",
                   "global_batch": nr, "parallelism": "none (1 GPU)"},
        "bfs": {"gteps": round(bfs_edges / (t_bfs / 1e3) / 1e9, 2), "ms_per_root": round(t_bfs / nr, 4),
                "hbm_gbs_algorithmic": round(bfs_bytes / (t_bfs / 1e3) / 1e9, 1),
                "graph500_undirected_gteps": round(bfs_edges / 2 / (t_bfs / 1e3) / 1e9, 2)},
        "sssp": {"gteps": round(sssp_edges / (t_sssp / 1e3) / 1e9, 2), "ms_per_root": round(t_sssp / nr, 4),
                 "supersteps_per_root": round(ss.get("supersteps", 0) / nr, 1),
                 "work_efficiency": round(ss.get("relaxations", 0) / max(sssp_edges, 1), 3)},
        "pagerank": {"gteps": round(pr_edges / (t_pr / 1e3) / 1e9, 2),
                     "ms_per_iter": round(t_pr / args.pr_iters, 4),
                     "hbm_gbs_algorithmic": round(pr_bytes_iter * args.pr_iters / (t_pr / 1e3) / 1e9, 1)},
        "roofline": dict(roofs[dominant], kernel=dominant) if dominant else None,
        "kernels": roofs,
        "tuning": {"source": tuning_used, "values": tg.partition_info(P)["tuning"]},
        "host_wall_s": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        units = {"bfs": bfs_edges, "sssp": sssp_edges, "pr": pr_edges}
        print("[bench] timing the oracle on the host (bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, w, roots, args.pr_iters, units)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
