"""Hybrid split (one GPU partition + one host-thread partition exchanging
reduced boundary messages each superstep) against the oracle: results must
equal the single-partition definitions exactly (BFS, SSSP) or within the
PageRank and BC tolerances, for every strategy and CPU edge share."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

SMALL_BINS = {"hub_min_deg": 300, "block_min_deg": 100, "wave_min_deg": 24, "g16_min_deg": 6,
              "g4_min_deg": 2, "hub_chunk": 256}


def pr_rel_l1(got, ref):
    return float(np.abs(got.astype(np.float64) - ref).sum() / np.abs(ref).sum())


def bc_close(got, ref):
    got = got.astype(np.float64)
    tol = 1e-4 * np.abs(ref) + 1e-6 * max(np.abs(ref).max(), 1.0)
    return np.all(np.abs(got - ref) <= tol)


@pytest.fixture(scope="module", params=["sym", "dir"])
def graph(request):
    g = graphgen.rmat(12, symmetrize=(request.param == "sym"))
    return g, graphgen.weights(g, seed=6)


@pytest.mark.parametrize("strategy", ["high", "low", "rand"])
@pytest.mark.parametrize("alpha", [0.1, 0.5])
def test_hybrid_matches_oracle(gpu, graph, strategy, alpha):
    g, w = graph
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, w, symmetric=g.symmetric)
    P = gpu.partition_by_degree(G, strategy, alpha, seed=11, tuning=SMALL_BINS)
    info = P.info()
    assert info["cpu_edges"] + info["gpu_edges"] + info["boundary_edges"] == g.nnz
    deg = np.diff(g.offsets)
    # a root on each side: the max-degree vertex and the min-degree non-isolated one
    roots = [graphgen.max_degree_vertex(g), int(np.argmin(np.where(deg > 0, deg, 1 << 30)))]
    roots += graphgen.sample_roots(g, 2, seed=4).tolist()
    lev = gpu.bfs(P, roots).cpu().numpy()
    st = gpu.tg_last_stats()
    # bitmaps: at most one bit per GPU-to-host slot and one per host vertex
    # (its frontier) per superstep
    words = (info["outbox_gpu_to_cpu"] + 31) // 32 + (info["cpu_vertices"] + 31) // 32
    assert st["exchange_bytes"] <= 4 * words * st["supersteps"]
    dist = gpu.sssp(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(lev[i], oracle.bfs(g.offsets, g.cols, r)), (strategy, alpha, r)
        assert np.array_equal(dist[i], oracle.sssp(g.offsets, g.cols, w, r)), (strategy, alpha, r)
    for mode in ("uniform", "drop"):
        rank = gpu.pagerank(P, 0.85, 10, mode).cpu().numpy()
        assert pr_rel_l1(rank, oracle.pagerank(g.offsets, g.cols, 0.85, 10, mode)) <= 1e-5
    st = gpu.tg_last_stats()
    assert st["supersteps"] == 10
    # 4 bytes per GPU-to-host slot and per host vertex, every iteration
    assert st["exchange_bytes"] == 4 * 10 * (info["outbox_gpu_to_cpu"] + info["cpu_vertices"])
    # Brandes BC with sigma and delta messages (sources on both sides)
    got = gpu.bc(P, roots).cpu().numpy()
    assert bc_close(got, oracle.bc(g.offsets, g.cols, roots)), (strategy, alpha)


def test_partition_statistics(gpu):
    g = graphgen.rmat(14)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True)
    E = g.nnz
    for alpha in (0.1, 0.3, 0.5):
        hi = gpu.partition_by_degree(G, "high", alpha).info()
        lo = gpu.partition_by_degree(G, "low", alpha).info()
        rd = gpu.partition_by_degree(G, "rand", alpha, seed=3).info()
        for inf in (hi, lo, rd):
            assert inf["cpu_vertices"] + inf["gpu_vertices"] == g.n
            assert inf["beta_reduced"] <= inf["beta_raw"]
        # HIGH holds its edge share with far fewer vertices than LOW or RAND (section 6.3.2)
        assert hi["cpu_vertices"] * 10 < rd["cpu_vertices"]
        assert hi["cpu_vertices"] * 10 < lo["cpu_vertices"]


def test_hybrid_rejects_unsupported(gpu):
    g = graphgen.rmat(10)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True)
    P = gpu.partition_by_degree(G, "high", 0.3)
    for call in (lambda: gpu.bc_batched(P, [0]), lambda: gpu.cc(P)):
        with pytest.raises(gpu.TGError) as ei:
            call()
        assert ei.value.code == gpu.TG_EUNSUPPORTED
    with pytest.raises(gpu.TGError):
        gpu.partition_by_degree(G, "high", 0.999999)


@pytest.mark.skip(reason="a GPU run that included this test (with an outbox variant since removed) ended in a "
                         "device fault whose cause was not found; kept off the GPU until one is shown")
@pytest.mark.parametrize("strategy", ["rand", "low"])
def test_hybrid_deep_search(gpu, strategy):
    """A 48x48 grid plus a directed tail: about a hundred supersteps with
    messages crossing both ways, several roots in a row on one partition (the
    per-search message state must start clean), and vertices no root reaches."""
    side = 48
    ids = np.arange(side * side).reshape(side, side)
    src = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    dst = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    grid = graphgen.from_edges(side * side + 40, src, dst, symmetrize=True)
    # a directed chain hanging off the corner, and 20 vertices never reached
    tail_src = np.concatenate([[side * side - 1], side * side + np.arange(19)])
    tail_dst = side * side + np.arange(20)
    s = np.concatenate([np.repeat(np.arange(grid.n), np.diff(grid.offsets)), tail_src])
    d = np.concatenate([grid.cols, tail_dst])
    g = graphgen.from_edges(grid.n, s, d, symmetrize=False)
    w = graphgen.weights(g, seed=8)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, w, symmetric=False)
    P = gpu.partition_by_degree(G, strategy, 0.4, seed=5, tuning=SMALL_BINS)
    roots = [0, side * side - 1, side * (side // 2) + side // 3, side * side + 3]
    lev = gpu.bfs(P, roots).cpu().numpy()
    dist = gpu.sssp(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(lev[i], oracle.bfs(g.offsets, g.cols, r)), (strategy, r)
        assert np.array_equal(dist[i], oracle.sssp(g.offsets, g.cols, w, r)), (strategy, r)
    inf = np.iinfo(np.int32).max
    assert (lev[0] == inf).sum() == 20 and lev[0][lev[0] < inf].max() >= 90


@pytest.mark.parametrize("strategy", ["rand", "low", "high"])
def test_hybrid_long_path(gpu, strategy):
    """A path of 1500 vertices with a few chords, split so that the frontier
    crosses the boundary at most supersteps: hundreds of supersteps with
    one-vertex frontiers, each side's outbox sending a slot at most once
    (BFS, BC) or again after every improvement (SSSP)."""
    n = 1500
    src = np.concatenate([np.arange(n - 1), [0, 100, 700]])
    dst = np.concatenate([np.arange(1, n), [50, 400, 1499]])
    g = graphgen.from_edges(n, src, dst, symmetrize=True)
    w = graphgen.weights(g, seed=9)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, w, symmetric=True)
    P = gpu.partition_by_degree(G, strategy, 0.5, seed=3)
    roots = [0, 777, n - 1]
    lev = gpu.bfs(P, roots).cpu().numpy()
    assert gpu.tg_last_stats()["supersteps"] > 300
    dist = gpu.sssp(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(lev[i], oracle.bfs(g.offsets, g.cols, r)), (strategy, r)
        assert np.array_equal(dist[i], oracle.sssp(g.offsets, g.cols, w, r)), (strategy, r)
    assert bc_close(gpu.bc(P, roots[:2]).cpu().numpy(), oracle.bc(g.offsets, g.cols, roots[:2]))
