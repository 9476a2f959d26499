"""Host logic of the autotuner and of the bench's reuse of measured traffic
(no GPU): candidate validity, the JSON cache, the acceptance rule of the
coordinate descent on a synthetic cost, and the digest that ties a traffic
figure to the kernel sources and the cached launch shapes."""
import json
import os
import shutil

import bench
from paper_1312_3018_amd import autotune


def test_valid_requires_ordered_thresholds():
    assert autotune.valid(autotune.DEFAULTS)
    bad = dict(autotune.DEFAULTS, wave_min_deg=autotune.DEFAULTS["block_min_deg"] + 1)
    assert not autotune.valid(bad)
    assert not autotune.valid(dict(autotune.DEFAULTS, g4_min_deg=50))
    assert not autotune.valid(dict(autotune.DEFAULTS, hub_chunk=128))
    # equal neighbouring thresholds leave a bin empty, which is allowed
    assert autotune.valid(dict(autotune.DEFAULTS, block_min_deg=autotune.DEFAULTS["hub_min_deg"]))


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "cache.json")
    assert autotune.load_cached("k1", path) is None
    r1 = {"config": dict(autotune.DEFAULTS, hub_chunk=1024), "initial_ms": {"all": 2.0},
          "final_ms": {"all": 1.0}, "trials": 3, "log": [{"key": "hub_chunk"}]}
    autotune.save_cached("k1", r1, path)
    autotune.save_cached("k2", dict(r1, config={"hub_chunk": 2048}), path)
    assert autotune.load_cached("k1", path)["hub_chunk"] == 1024
    assert autotune.load_cached("k2", path) == {"hub_chunk": 2048}
    assert "log" not in json.load(open(path))["k1"]  # the trial log is not cached
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune.load_cached("k1", path) is None
    autotune.save_cached("k3", r1, path)  # a corrupt cache is replaced
    assert autotune.load_cached("k3", path)["hub_chunk"] == 1024


def _cost(gains):
    """Synthetic times: 100 ms per family minus the listed gains (ms) for
    the keys whose value matches; records every configuration measured."""
    seen = []

    def f(cfg, fam):
        assert autotune.valid(cfg)
        seen.append((dict(cfg), fam))
        return 100.0 - sum(g for (k, v, fams), g in gains.items() if cfg[k] == v and fam in fams)
    return f, seen


def test_search_keeps_only_gains_beyond_the_margin():
    gains = {("hub_chunk", 1024, ("all",)): 5.0,           # 5%: taken
             ("sssp_grid", 4096, ("sssp",)): 1.0,          # 1%: below the 2% margin
             ("bfs_alpha", 32, ("bfs",)): 3.0,             # 3%: taken
             ("pr_grid", 512, ("all", "bfs", "sssp")): 9}  # pr_grid is scored on "pr" only
    f, seen = _cost(gains)
    res = autotune.tune(None, [], None, start={}, measure_fn=f)
    cfg = res["config"]
    assert cfg["hub_chunk"] == 1024 and cfg["bfs_alpha"] == 32
    assert cfg["sssp_grid"] == autotune.DEFAULTS["sssp_grid"]
    assert cfg["pr_grid"] == autotune.DEFAULTS["pr_grid"]
    assert res["final_ms"]["all"] == 95.0 and res["final_ms"]["bfs"] == 97.0
    assert res["initial_ms"] == {"all": 100.0, "bfs": 100.0, "pr": 100.0, "sssp": 100.0}
    # one trial per candidate value that differs from the current one (after
    # hub_chunk moves to 1024, the default 4096 is a candidate again)
    taken = {("hub_chunk", 1024), ("bfs_alpha", 32)}
    expect = 0
    for k, vals in autotune.SPACE.items():
        cur = autotune.DEFAULTS[k]
        for v in vals:
            if v != cur:
                expect += 1
                cur = v if (k, v) in taken else cur
    assert res["trials"] == expect
    # every candidate was scored on its own key's family
    for cfg_m, fam in seen[4:]:
        changed = [k for k in autotune.SPACE if cfg_m[k] != autotune.DEFAULTS[k] and
                   not (k == "hub_chunk" and cfg_m[k] == 1024) and not (k == "bfs_alpha" and cfg_m[k] == 32)]
        assert len(changed) <= 1
        if changed:
            assert autotune.FAMILY[changed[0]] == fam


def test_search_skips_invalid_candidates():
    f, seen = _cost({})
    start = {"hub_min_deg": 8192, "block_min_deg": 4096}
    res = autotune.tune(None, [], None, start=start, measure_fn=f)
    assert res["config"]["block_min_deg"] == 4096
    assert all(c["hub_min_deg"] >= c["block_min_deg"] for c, _ in seen)
    assert not any(c["hub_min_deg"] == 2048 for c, _ in seen)


def test_traffic_is_tied_to_sources_and_tuning(tmp_path, monkeypatch):
    # a copy of the files the digests read, so the real tree is untouched
    src = os.path.join(bench.ROOT, "paper_1312_3018_amd")
    os.makedirs(tmp_path / "paper_1312_3018_amd" / "csrc")
    os.makedirs(tmp_path / "profiles")
    files = sorted({f for fs in bench.KERNEL_FILES.values() for f in fs})
    for f in files:
        shutil.copy(os.path.join(src, "csrc", f), tmp_path / "paper_1312_3018_amd" / "csrc" / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert all("../tuning_cache.json" in fs for fs in bench.KERNEL_FILES.values())
    dig = bench.kernel_sources_digest(bench.KERNEL_FILES["sssp_relax"])
    with open(tmp_path / "profiles" / "traffic.json", "w") as fh:
        json.dump({"w": {"sssp_relax": {"bytes_per_launch": 123, "sources": dig}}}, fh)
    assert bench.load_traffic("sssp_relax", "w") == 123
    assert bench.load_traffic("sssp_relax", "other") is None
    with open(tmp_path / "paper_1312_3018_amd" / "tuning_cache.json", "a") as fh:
        fh.write("\n")  # new launch shapes: the stored figure no longer applies
    assert bench.load_traffic("sssp_relax", "w") is None


def test_traffic_from_counter_csvs(tmp_path):
    """traffic.json rows from rocprofv3 counter CSVs: per-kernel means over
    launches, summed over a bench kernel's kernels, scaled by the copy
    calibration; the L2 hit rate from the hit/miss pass."""
    rows = {"fetch": "FETCH_SIZE", "write": "WRITE_SIZE"}
    names = {"sssp": ["k_sssp_relax<true, 1>(int const*)", "k_sssp_relax<true, 2>(int const*)"],
             "ssspp": ["k_sssp_pull_heavy(Plan const*)"],
             "pr": ["k_pr_rows<true, int, 8>(Args)", "k_pr_long<true>(Args)", "k_pr_combine(x)", "k_pr_dsum(y)"],
             "bfs": ["k_bfs_step<int>(a)"]}
    for algo, kernels in names.items():
        for kind in ("fetch", "write", "hit"):
            d = tmp_path / f"{algo}_{kind}"
            d.mkdir()
            lines = ["Kernel_Name,Counter_Name,Counter_Value"]
            for i, k in enumerate(kernels):
                if kind == "hit":
                    lines += [f'"{k}",TCC_HIT_sum,30', f'"{k}",TCC_MISS_sum,10']
                else:  # two launches per kernel: 100 and 300 KiB, mean 200
                    lines += [f'"{k}",{rows[kind]},100', f'"{k}",{rows[kind]},300']
            (d / "run_counter_collection.csv").write_text("\n".join(lines) + "\n")
    t = bench.traffic_from(str(tmp_path))["rmat24"]
    kib = 200 * 1024
    assert t["sssp_relax"]["fetch_bytes"] == round(kib * bench.FETCH_SCALE)
    assert t["sssp_relax"]["write_bytes"] == round(kib * bench.WRITE_SCALE)
    assert t["sssp_relax"]["launches_sampled"] == 4  # pooled: two launches of each variant
    assert t["pr_gather"]["fetch_bytes"] == round(4 * kib * bench.FETCH_SCALE)
    assert t["bfs_step"]["write_bytes"] == kib
    assert t["sssp_pull"]["fetch_bytes"] == round(kib * bench.FETCH_SCALE)
    assert all(r["l2_hit_rate"] == 0.75 for r in t.values())
    assert t["sssp_relax"]["sources"] == bench.kernel_sources_digest(bench.KERNEL_FILES["sssp_relax"])
