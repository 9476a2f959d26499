"""Autotuner for the degree-bin thresholds and launch shapes of libtg.

Coordinate descent over a small discrete space: each key is swept in turn
with the others fixed, and a value is kept when it lowers the measured time
of the kernels it affects.  Bin thresholds and the hub chunk affect every
algorithm and are scored on the whole step (BFS + SSSP + PageRank); the
PageRank and BFS launch-shape keys are scored on their own algorithm.
Candidates are applied with partition_retune (no rebuild); times come from
HIP events on the launching stream.  Results are cached as JSON keyed by the
device architecture and a coarse graph signature.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Dict, List, Optional, Sequence

from . import bfs, pagerank, partition_info, partition_retune, sssp

DEFAULTS = {
    "hub_min_deg": 8192, "block_min_deg": 512, "wave_min_deg": 48, "g16_min_deg": 12, "g4_min_deg": 3,
    "hub_chunk": 4096, "pr_lds_verts": 40960, "pr_grid": 256, "bfs_lds_words": 4096, "bfs_grid": 2048,
    "bfs_lds_min_vblocks": 4096, "sssp_delta": 32, "sssp_lds_verts": 0, "sssp_grid": 2048, "pr_xcd": 1,
    "pr_rows": 512, "bfs_do": 1, "bfs_alpha": 14, "bfs_beta": 24, "sssp_xcd": 0,
    "bfs_lanes": 2, "bfs_td_grid": 1024, "bfs_bu_grid": 4096, "sssp_lanes": 4, "sssp_pull": 0, "sssp_packed": 1, "sssp_ring": 1, "sssp_split": 1, "sssp_hpull": 100,
    "bfs_graph": 0,
}

SPACE = {
    "hub_min_deg": [2048, 4096, 8192, 16384, 65536],
    "block_min_deg": [256, 512, 1024, 2048],
    "wave_min_deg": [24, 48, 96, 192],
    "g16_min_deg": [6, 12, 24],
    "g4_min_deg": [2, 3, 5],
    "hub_chunk": [1024, 2048, 4096, 8192],
    "pr_xcd": [0, 1],
    "pr_rows": [256, 512],
    "pr_lds_verts": [0, 8192, 16384, 24576, 32768, 40960],
    "pr_grid": [256, 512, 1024],
    "bfs_td_grid": [512, 1024, 2048],
    "bfs_bu_grid": [2048, 4096, 8192],
    "bfs_lanes": [1, 2, 3, 4],
    "bfs_graph": [0, 1],
    "bfs_alpha": [4, 14, 32, 64],
    "bfs_beta": [8, 24, 64],
    "sssp_delta": [0, 16, 24, 32, 48, 64, 128],
    "sssp_lanes": [1, 2, 3, 4, 6, 8],
    "sssp_pull": [0, 50, 70],
    "sssp_packed": [0, 1],
    "sssp_ring": [0, 1],
    "sssp_split": [0, 1],
    "sssp_hpull": [0, 50, 100, 200],
    "sssp_lds_verts": [0, 2048, 4096, 8192],
    "sssp_grid": [1024, 2048, 4096, 16384],
    "sssp_xcd": [0, 1],
}

FAMILY = {k: "all" for k in ("hub_min_deg", "block_min_deg", "wave_min_deg", "g16_min_deg", "g4_min_deg",
                             "hub_chunk")}
FAMILY.update({"pr_xcd": "pr", "pr_rows": "pr", "pr_lds_verts": "pr", "pr_grid": "pr", "bfs_td_grid": "bfs",
               "bfs_bu_grid": "bfs", "bfs_lanes": "bfs", "bfs_graph": "bfs", "bfs_alpha": "bfs", "bfs_beta": "bfs",
               "sssp_delta": "sssp", "sssp_lds_verts": "sssp", "sssp_lanes": "sssp", "sssp_pull": "sssp", "sssp_packed": "sssp", "sssp_ring": "sssp", "sssp_split": "sssp", "sssp_hpull": "sssp",
               "sssp_grid": "sssp", "sssp_xcd": "sssp"})

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def valid(cfg: Dict[str, int]) -> bool:
    t = [cfg["hub_min_deg"], cfg["block_min_deg"], cfg["wave_min_deg"], cfg["g16_min_deg"], cfg["g4_min_deg"]]
    return all(a >= b for a, b in zip(t, t[1:])) and cfg["hub_chunk"] >= 256


def graph_key(part, arch: str = "gfx950") -> str:
    """Architecture plus a coarse signature: log2(V), rounded average degree,
    symmetry.  Graphs of one generator family and size share an entry."""
    info = partition_info(part)
    V, E = info["V"], info["E"]
    avg = E / max(V, 1)
    return f"{arch}:V2^{round(math.log2(max(V, 1)))}:deg{round(avg)}:{'sym' if info['symmetric'] else 'dir'}"


def _timed(fn) -> float:
    import torch
    s = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b)


def measure(part, cfg, roots, sssp_roots, pr_iters, family: str, bufs, repeats: int = 2) -> float:
    partition_retune(part, cfg)
    lev, dist, rank = bufs
    best = math.inf
    for _ in range(repeats):
        ms = 0.0
        if family in ("all", "bfs"):
            ms += _timed(lambda: bfs(part, roots, lev))
        if family in ("all", "sssp") and sssp_roots is not None and len(sssp_roots):
            ms += _timed(lambda: sssp(part, sssp_roots, dist))
        if family in ("all", "pr"):
            ms += _timed(lambda: pagerank(part, 0.85, pr_iters, "uniform", rank))
        best = min(best, ms)
    return best


def tune(part, roots: Sequence[int], sssp_roots: Optional[Sequence[int]] = None, pr_iters: int = 5,
         start: Optional[Dict[str, int]] = None, rounds: int = 1,
         log: Callable[[str], None] = lambda s: None,
         measure_fn: Optional[Callable[[Dict[str, int], str], float]] = None) -> Dict[str, object]:
    """Coordinate descent from `start` (or DEFAULTS).  `measure_fn(cfg,
    family)` replaces the timed runs (no device buffers are allocated then)."""
    if measure_fn is None:
        import torch
        V = part.n
        lev = torch.empty((len(roots), V), dtype=torch.int32, device="cuda")
        n_ss = 0 if sssp_roots is None else len(sssp_roots)
        dist = torch.empty((max(n_ss, 1), V), dtype=torch.int32, device="cuda")
        rank = torch.empty((V,), dtype=torch.float32, device="cuda")
        bufs = (lev, dist, rank)
        measure_fn = lambda c, f: measure(part, c, roots, sssp_roots, pr_iters, f, bufs)
    cfg = dict(DEFAULTS)
    if start:
        cfg.update(start)
    trials: List[dict] = []
    t0 = time.perf_counter()
    fams = ("all", "bfs", "pr", "sssp")
    base = {f: measure_fn(cfg, f) for f in fams}
    initial = dict(base)
    for r in range(rounds):
        for key, values in SPACE.items():
            fam = FAMILY[key]
            for v in values:
                if v == cfg[key]:
                    continue
                cand = dict(cfg, **{key: v})
                if not valid(cand):
                    continue
                ms = measure_fn(cand, fam)
                trials.append({"key": key, "value": v, "family": fam, "ms": ms})
                if ms < base[fam] * 0.98:
                    log(f"[autotune] {key}={v}: {base[fam]:.3f} -> {ms:.3f} ms ({fam})")
                    cfg = cand
                    base[fam] = ms
                    # a shared key changes the per-family baselines too
                    if fam == "all":
                        for f in fams[1:]:
                            base[f] = measure_fn(cfg, f)
    if part is not None:
        partition_retune(part, cfg)
    return {"config": cfg, "initial_ms": initial, "final_ms": base, "trials": len(trials),
            "seconds": round(time.perf_counter() - t0, 1), "log": trials}


def load_cached(key: str, path: str = CACHE) -> Optional[Dict[str, int]]:
    if not os.path.exists(path):
        return None
    try:
        return json.load(open(path)).get(key, {}).get("config")
    except (OSError, ValueError):
        return None


def save_cached(key: str, result: Dict[str, object], path: str = CACHE) -> None:
    data = {}
    if os.path.exists(path):
        try:
            data = json.load(open(path))
        except ValueError:
            data = {}
    data[key] = {"config": result["config"], "initial_ms": result["initial_ms"],
                 "final_ms": result["final_ms"], "trials": result["trials"]}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
