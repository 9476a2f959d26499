"""The performance model of section 3 as the bench evaluates it (host logic,
no GPU): Equation 4's limits and the achieved-speedup definition on
synthetic measurements with known answers."""
import math

import bench


def row(strategy, alpha, *, E, beta, bfs_ms, pr_ms, host_rate, c_bytes):
    # a split whose host threads process alpha*E local edges at host_rate
    # edges/s; the PageRank exchange moves c_bytes bytes per second of copy
    cpu_edges = alpha * E
    return {"strategy": strategy, "alpha": alpha, "cpu_edges": int(cpu_edges), "beta_reduced": beta,
            "bfs_cpu_edges": int(cpu_edges), "bfs_cpu_ms": cpu_edges / host_rate * 1e3,
            "bfs_edges": E, "bfs_ms": bfs_ms, "pr_exchange_bytes": int(c_bytes), "pr_exchange_ms": 1000.0,
            "pr_cpu_edges": int(cpu_edges), "pr_cpu_ms": cpu_edges / host_rate * 1e3, "pr_ms_per_iter": pr_ms}


def test_model_matches_equation_4():
    E, r, c_bytes = 10**9, 2e9, 4e9  # c = 1e9 messages/s of 4 bytes
    rows = [{"strategy": "high", "alpha": 0.0, "bfs_cpu_ms": 0}]
    # hybrid time = exactly the host's share of the host-only time: the
    # achieved speedup is 1/alpha, the model's beta = 0 limit
    for a in (0.1, 0.25, 0.5):
        t = a * E / r * 1e3
        rows.append(row("high", a, E=E, beta=0.0, bfs_ms=t, pr_ms=t, host_rate=r, c_bytes=c_bytes))
    m = bench.hybrid_model(rows, E, lambda s: None)
    assert m["r_cpu_from"] == "high alpha=0.5"
    assert math.isclose(m["r_cpu_eps"]["bfs"], r, rel_tol=1e-6)
    assert math.isclose(m["c_msgs_per_s"], 1e9, rel_tol=1e-6)
    for p in m["points"]:
        for alg in ("bfs", "pagerank"):
            assert math.isclose(p[alg]["predicted"], 1 / p["alpha"], rel_tol=1e-3)
            assert math.isclose(p[alg]["achieved"], 1 / p["alpha"], rel_tol=1e-3)
            assert abs(p[alg]["error"]) < 1e-3
    assert m["bfs"]["correlation_high"] > 0.999


def test_model_communication_term():
    # beta * r_cpu / c adds to alpha in the denominator (Equation 4)
    E, r, c_bytes, beta = 10**9, 4e9, 4e9, 0.05
    rows = [row("high", 0.2, E=E, beta=beta, bfs_ms=100.0, pr_ms=100.0, host_rate=r, c_bytes=c_bytes)]
    m = bench.hybrid_model(rows, E, lambda s: None)
    p = m["points"][0]
    expect = 1.0 / (beta * r / 1e9 + 0.2)
    assert math.isclose(p["bfs"]["predicted"], expect, rel_tol=1e-3)
    # achieved: host-only time E / r over the measured 100 ms
    assert math.isclose(p["bfs"]["achieved"], (E / r) / 0.1, rel_tol=1e-3)
    assert m["bfs"]["correlation_high"] is None  # one point: undefined


def test_model_without_splits():
    assert bench.hybrid_model([{"strategy": "high", "alpha": 0.0, "bfs_cpu_ms": 0}], 10, lambda s: None) is None


def test_serve_solo_rule(monkeypatch):
    """The serving bench takes a lane the way the server's default rule
    serves it: single searches only on graphs at or above the vertex floor
    whose largest out-degree is at least 16 times the mean (host logic)."""
    import numpy as np

    import graphgen
    n = 2000
    star = graphgen.from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n), symmetrize=True)
    ring = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n, symmetrize=True)
    assert not bench.serve_solo(star)  # below the 2^22-vertex floor
    monkeypatch.setattr(bench, "SERVE_SOLO_MIN_VERTICES", 0)
    assert bench.serve_solo(star)  # skew about 1000
    assert not bench.serve_solo(ring)  # every degree 2: skew 1
