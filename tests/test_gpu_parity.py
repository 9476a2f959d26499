"""GPU parity: the HIP path (through the C ABI) against the oracle on the same
seeded inputs.  BFS levels and SSSP distances are bit-exact; PageRank within
1e-5 relative L1 of the fp64 oracle; betweenness within 1e-4 relative per
vertex (plus 1e-6 of the largest score, for near-zero scores)."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

INF = oracle.INF
# small thresholds so that tiny graphs exercise every degree bin, including
# multi-chunk hubs
SMALL_BINS = {"hub_min_deg": 300, "block_min_deg": 100, "wave_min_deg": 24, "g16_min_deg": 6,
              "g4_min_deg": 2, "hub_chunk": 256, "pr_lds_verts": 100, "pr_grid": 7,
              "bfs_lds_words": 16, "bfs_grid": 5, "bfs_lds_min_vblocks": 0,
              "sssp_delta": 64, "sssp_lds_verts": 100, "sssp_grid": 6, "pr_rows": 256}
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(tg, g, weights=None, tuning=None, **kw):
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, weights, symmetric=g.symmetric)
    return tg.partition_by_degree(G, tuning=tuning, **kw)


def pr_rel_l1(got, ref):
    return float(np.abs(got.astype(np.float64) - ref).sum() / np.abs(ref).sum())


def bc_close(got, ref):
    got = got.astype(np.float64)
    tol = 1e-4 * np.abs(ref) + 1e-6 * max(np.abs(ref).max(), 1.0)
    return np.all(np.abs(got - ref) <= tol)


def six(tg, tuning=None):
    d = json.load(open(os.path.join(GOLD, "six_vertex.json")))
    e = np.array(d["undirected_edges"])
    g = graphgen.from_edges(6, e[:, 0], e[:, 1], symmetrize=True)
    wmap = {}
    for a, b, w in d["undirected_edges"]:
        wmap[(a, b)] = wmap[(b, a)] = w
    w = np.array([wmap[(u, int(v))] for u in range(6) for v in g.cols[g.offsets[u]:g.offsets[u + 1]]],
                 dtype=np.int32)
    return d, g, w, load(tg, g, w, tuning)


# ------------------------------------------------------------- hand-worked

def test_six_vertex_example(gpu):
    d, g, w, P = six(gpu)
    assert gpu.bfs(P, [0]).cpu().numpy()[0].tolist() == d["bfs_from_0"]
    assert gpu.sssp(P, [0, 3]).cpu().numpy().tolist() == [d["sssp_from_0"], d["sssp_from_3"]]
    assert np.allclose(gpu.bc(P, [0]).cpu().numpy(), d["bc_source_0"], atol=1e-6)
    assert np.allclose(gpu.bc(P, range(6)).cpu().numpy(), d["bc_all_sources"], atol=1e-5)
    r1 = gpu.pagerank(P, 0.85, 1).cpu().numpy()
    assert np.allclose(r1, [a / b for a, b in d["pagerank_r1_fraction"]], rtol=1e-6)


# ----------------------------------------------------- RMAT-14 full parity

@pytest.fixture(scope="module")
def rmat14():
    g = graphgen.rmat(14)
    return g, graphgen.weights(g, seed=2)


@pytest.mark.parametrize("tuning", [None, SMALL_BINS])
def test_rmat14_bfs_pagerank(gpu, rmat14, tuning):
    g, w = rmat14
    P = load(gpu, g, w, tuning)
    root = graphgen.max_degree_vertex(g)
    roots = [root] + graphgen.sample_roots(g, 5, seed=3).tolist()
    lev = gpu.bfs(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(lev[i], oracle.bfs(g.offsets, g.cols, r)), f"root {r}"
    rank = gpu.pagerank(P, 0.85, 10).cpu().numpy()
    ref = oracle.pagerank(g.offsets, g.cols, 0.85, 10)
    assert pr_rel_l1(rank, ref) <= 1e-5
    assert abs(rank.astype(np.float64).sum() - 1.0) < 1e-5


@pytest.mark.parametrize("tuning", [None, SMALL_BINS])
def test_rmat14_sssp(gpu, rmat14, tuning):
    g, w = rmat14
    P = load(gpu, g, w, tuning)
    roots = graphgen.sample_roots(g, 6, seed=5)
    dist = gpu.sssp(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(dist[i], oracle.sssp(g.offsets, g.cols, w, r)), f"root {r}"


@pytest.mark.parametrize("tuning", [None, SMALL_BINS])
def test_rmat12_bc(gpu, tuning):
    g = graphgen.rmat(12)
    P = load(gpu, g, None, tuning)
    srcs = graphgen.sample_roots(g, 8, seed=7)
    got = gpu.bc(P, srcs).cpu().numpy()
    ref = oracle.bc(g.offsets, g.cols, srcs)
    assert bc_close(got, ref)


@pytest.mark.parametrize("lanes", [1, 3, 4])
def test_bfs_lanes(gpu, rmat14, lanes):
    """Several BFS searches in flight (a workspace and stream each, served in
    turn): every row equals the oracle, with more roots than lanes and one
    root repeated."""
    g, w = rmat14
    P = load(gpu, g, w, {"bfs_lanes": lanes})
    roots = graphgen.sample_roots(g, 9, seed=31).tolist()
    roots.append(roots[2])
    lev = gpu.bfs(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(lev[i], oracle.bfs(g.offsets, g.cols, r)), (lanes, r)
    assert gpu.tg_last_stats()["lanes"] == min(lanes, len(roots))


@pytest.mark.parametrize("delta", [1, 300, 1 << 20])
def test_sssp_near_far_thresholds(gpu, rmat14, delta):
    g, w = rmat14
    P = load(gpu, g, w, {"sssp_delta": delta, "sssp_lds_verts": 4096})
    roots = graphgen.sample_roots(g, 3, seed=15)
    dist = gpu.sssp(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(dist[i], oracle.sssp(g.offsets, g.cols, w, r))


def test_bfs_parents_valid(gpu, rmat14):
    g, w = rmat14
    P = load(gpu, g, w, SMALL_BINS)
    root = graphgen.max_degree_vertex(g)
    lev, par = gpu.bfs(P, [root], want_parents=True)
    lev, par = lev.cpu().numpy()[0], par.cpu().numpy()[0]
    assert np.array_equal(lev, oracle.bfs(g.offsets, g.cols, root))
    assert par[root] == root
    reach = (lev != INF) & (np.arange(g.n) != root)
    assert np.all(par[lev == INF] == -1)
    v = np.nonzero(reach)[0]
    p = par[v]
    assert np.all(lev[p] == lev[v] - 1)
    for a, b in zip(p[:2000], v[:2000]):
        assert b in g.cols[g.offsets[a]:g.offsets[a + 1]]


# ------------------------------------------------------------ directed graphs

@pytest.mark.parametrize("tuning", [None, SMALL_BINS])
def test_directed_rmat12_all(gpu, tuning):
    g = graphgen.rmat(12, symmetrize=False)
    w = graphgen.weights(g, seed=4)
    P = load(gpu, g, w, tuning)
    roots = graphgen.sample_roots(g, 3, seed=9)
    lev = gpu.bfs(P, roots).cpu().numpy()
    dist = gpu.sssp(P, roots).cpu().numpy()
    for i, r in enumerate(roots):
        assert np.array_equal(lev[i], oracle.bfs(g.offsets, g.cols, r))
        assert np.array_equal(dist[i], oracle.sssp(g.offsets, g.cols, w, r))
    for mode in ("uniform", "drop"):
        rank = gpu.pagerank(P, 0.85, 20, mode).cpu().numpy()
        assert pr_rel_l1(rank, oracle.pagerank(g.offsets, g.cols, 0.85, 20, mode)) <= 1e-5
    got = gpu.bc(P, roots).cpu().numpy()
    assert bc_close(got, oracle.bc(g.offsets, g.cols, roots))


@pytest.mark.parametrize("xcd", [0, 1])
@pytest.mark.parametrize("rows", [256, 512])
def test_pagerank_variants(gpu, rmat14, xcd, rows):
    """Every PageRank gather variant (row blocks of each size, whole CSR or
    per-XCD source classes, hot table off/small/full) on a symmetric and a
    directed graph; row blocks of 256 edges split the hubs into many chunks."""
    g, w = rmat14
    gd = graphgen.rmat(12, symmetrize=False)
    for graph, iters in ((g, 10), (gd, 20)):
        for lds in (0, 100, 40960):
            tuning = {"pr_xcd": xcd, "pr_rows": rows, "pr_lds_verts": lds, "pr_grid": 64}
            P = load(gpu, graph, None, tuning)
            for mode in ("uniform", "drop"):
                rank = gpu.pagerank(P, 0.85, iters, mode).cpu().numpy()
                ref = oracle.pagerank(graph.offsets, graph.cols, 0.85, iters, mode)
                assert pr_rel_l1(rank, ref) <= 1e-5, (tuning, mode)
            again = gpu.pagerank(P, 0.85, iters, "drop").cpu().numpy()
            assert np.array_equal(again, rank)  # deterministic


@pytest.mark.parametrize("xcd", [0, 1])
@pytest.mark.parametrize("delta", [0, 64])
def test_sssp_variants(gpu, rmat14, xcd, delta):
    """SSSP with and without the per-XCD destination classes and the near/far
    step, with small degree thresholds (multi-chunk hubs whose class rows
    differ in length) and the defaults, on symmetric, directed, star and path
    graphs."""
    g, w = rmat14
    gd = graphgen.rmat(12, symmetrize=False)
    gs = graphgen.from_edges(20001, np.zeros(20000, dtype=int), np.arange(1, 20001), symmetrize=True)
    gp = graphgen.from_edges(700, np.arange(699), np.arange(1, 700), symmetrize=True)
    cases = [(g, w, graphgen.sample_roots(g, 3, seed=21).tolist()),
             (gd, graphgen.weights(gd, seed=4), graphgen.sample_roots(gd, 3, seed=22).tolist()),
             (gs, graphgen.weights(gs, seed=5), [0, 3]),
             (gp, graphgen.weights(gp, seed=6), [0, 350])]
    for tuning in ({"sssp_xcd": xcd, "sssp_delta": delta},
                   dict(SMALL_BINS, sssp_xcd=xcd, sssp_delta=delta, sssp_grid=3)):
        for graph, wt, roots in cases:
            P = load(gpu, graph, wt, tuning)
            dist = gpu.sssp(P, roots).cpu().numpy()
            for i, r in enumerate(roots):
                assert np.array_equal(dist[i], oracle.sssp(graph.offsets, graph.cols, wt, r)), (tuning, graph.n, r)


@pytest.mark.parametrize("ring,split,hpull", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 100), (1, 1, 100000)])
def test_sssp_bucket_ring(gpu, rmat14, ring, split, hpull):
    """The near/far step over a ring of bucket bitmaps (with and without
    the light/heavy split of each row, and, with ring = 0, over one far
    pile) gives the oracle's distances for bucket widths that need 3 to 12
    bitmaps with weights 1..255, and for widths 1 and 2 with weights 1..3
    (width 1: no light edges at all), on symmetric and directed graphs, a
    star and a path, with hub rows split into chunks, for several roots in a
    row on one partition.  With the split, a bucket's heavy edges are always
    pushed (hpull 0), pulled when the unsettled vertices hold fewer edges
    (100), or pulled almost always (100000; directed graphs always push)."""
    g, w = rmat14
    gd = graphgen.rmat(12, symmetrize=False)
    wd = graphgen.weights(gd, seed=4)
    w3 = (w % 3 + 1).astype(np.int32)  # 1..3, one value per undirected edge like w
    gs = graphgen.from_edges(20001, np.zeros(20000, dtype=int), np.arange(1, 20001), symmetrize=True)
    gp = graphgen.from_edges(700, np.arange(699), np.arange(1, 700), symmetrize=True)
    small = {"hub_min_deg": 300, "block_min_deg": 100, "wave_min_deg": 24, "g16_min_deg": 6, "g4_min_deg": 2,
             "hub_chunk": 256}
    cases = [(g, w, d, None) for d in (24, 32, 128)] + [(g, w, 24, small), (gd, wd, 32, None), (g, w3, 1, None),
                                                       (g, w3, 2, small), (gs, graphgen.weights(gs, seed=5), 32, small),
                                                       (gp, graphgen.weights(gp, seed=6), 16, None)]
    for graph, wt, delta, bins in cases:
        P = load(gpu, graph, wt, dict(bins or {}, sssp_delta=delta, sssp_ring=ring, sssp_split=split,
                                      sssp_hpull=hpull))
        roots = graphgen.sample_roots(graph, 3, seed=delta)
        dist = gpu.sssp(P, roots).cpu().numpy()
        for i, r in enumerate(roots):
            assert np.array_equal(dist[i], oracle.sssp(graph.offsets, graph.cols, wt, r)), (delta, graph.n, r)


@pytest.mark.parametrize("pr_lds_verts", [0, 40960])
@pytest.mark.parametrize("delta", [0, 64])
def test_sssp_pull(gpu, rmat14, delta, pr_lds_verts):
    """Pull supersteps (sssp_pull = 1: every superstep whose frontier holds
    more than 1% of the edges pulls) give the oracle's distances: with and
    without the LDS table of hot frontier distances, with the near/far step,
    on a symmetric R-MAT graph, a star whose hub row is split into chunks, a
    path, a directed graph (no in-edge weights: push only) and overflowing
    weights (TG_ERANGE as with push)."""
    g, w = rmat14
    gd = graphgen.rmat(12, symmetrize=False)
    gs = graphgen.from_edges(20001, np.zeros(20000, dtype=int), np.arange(1, 20001), symmetrize=True)
    gp = graphgen.from_edges(700, np.arange(699), np.arange(1, 700), symmetrize=True)
    cases = [(g, w, graphgen.sample_roots(g, 4, seed=23).tolist() + [graphgen.max_degree_vertex(g)]),
             (gd, graphgen.weights(gd, seed=4), graphgen.sample_roots(gd, 3, seed=22).tolist()),
             (gs, graphgen.weights(gs, seed=5), [0, 3]),
             (gp, graphgen.weights(gp, seed=6), [0, 350])]
    tuning = {"sssp_pull": 1, "sssp_delta": delta, "pr_lds_verts": pr_lds_verts}
    pulled = 0
    for graph, wt, roots in cases:
        P = load(gpu, graph, wt, tuning)
        dist = gpu.sssp(P, roots).cpu().numpy()
        pulled += gpu.tg_last_stats()["pull_supersteps"]
        for i, r in enumerate(roots):
            assert np.array_equal(dist[i], oracle.sssp(graph.offsets, graph.cols, wt, r)), (tuning, graph.n, r)
    assert pulled > 0
    # overflow: a path whose second edge cannot be added below INT32_MAX
    go = graphgen.from_edges(3, [0, 1], [1, 2], symmetrize=True)
    wo = np.full(go.nnz, 2**31 - 10, dtype=np.int32)
    with pytest.raises(gpu.TGError) as ei:
        gpu.sssp(load(gpu, go, wo, tuning), [0])
    assert ei.value.code == gpu.TG_ERANGE


def test_bfs_captured_chunks(gpu, rmat14):
    """Superstep chunks captured as HIP graphs and replayed: every replay
    (three calls of twelve roots on two lanes, with other work on the stream
    between them, then after a retune that forces a new capture) gives the
    oracle's levels."""
    g, w = rmat14
    roots = [graphgen.max_degree_vertex(g)] + graphgen.sample_roots(g, 11, seed=31).tolist()
    refs = [oracle.bfs(g.offsets, g.cols, r) for r in roots]
    P = load(gpu, g, w, {"bfs_graph": 1})
    for tuning in ({"bfs_graph": 1}, {"bfs_graph": 1, "bfs_alpha": 1000000, "bfs_beta": 1}):
        gpu.partition_retune(P, tuning)
        for rep in range(3):
            lev = gpu.bfs(P, roots).cpu().numpy()
            for i, r in enumerate(roots):
                assert np.array_equal(lev[i], refs[i]), (tuning, rep, r)
            gpu.sssp(P, roots[:2])
            gpu.pagerank(P, 0.85, 2)


def test_mapped_edges(gpu, rmat14):
    """Edge arrays kept in mapped host memory (read by the kernels over the
    host link): every algorithm gives the oracle's results on a symmetric and
    a directed graph, and the per-XCD class layouts (which would copy the
    edges to the device) stay off even when a retune asks for them."""
    g, w = rmat14
    gd = graphgen.rmat(12, symmetrize=False)
    wd = graphgen.weights(gd, seed=4)
    for graph, wt in ((g, w), (gd, wd)):
        P = load(gpu, graph, wt, {"mapped_edges": 1})
        assert gpu.partition_info(P)["tuning"]["mapped_edges"] == 1
        roots = [graphgen.max_degree_vertex(graph)] + graphgen.sample_roots(graph, 3, seed=41).tolist()
        for tuning in (None, {"mapped_edges": 1, "pr_xcd": 1, "sssp_xcd": 1, "sssp_pull": 1}):
            if tuning:
                gpu.partition_retune(P, tuning)
                t = gpu.partition_info(P)["tuning"]
                assert t["pr_xcd"] == 0 and t["sssp_xcd"] == 0 and t["sssp_pull"] == 0
            lev = gpu.bfs(P, roots).cpu().numpy()
            dist = gpu.sssp(P, roots).cpu().numpy()
            for i, r in enumerate(roots):
                assert np.array_equal(lev[i], oracle.bfs(graph.offsets, graph.cols, r)), (graph.n, r)
                assert np.array_equal(dist[i], oracle.sssp(graph.offsets, graph.cols, wt, r)), (graph.n, r)
            rank = gpu.pagerank(P, 0.85, 10).cpu().numpy()
            assert pr_rel_l1(rank, oracle.pagerank(graph.offsets, graph.cols, 0.85, 10)) <= 1e-5
            assert bc_close(gpu.bc(P, roots[:2]).cpu().numpy(), oracle.bc(graph.offsets, graph.cols, roots[:2]))
            assert np.array_equal(gpu.cc(P).cpu().numpy(), oracle.cc(graph.offsets, graph.cols))


DO_VARIANTS = [{"bfs_do": 0},                                   # top-down only
               {"bfs_alpha": 1000000, "bfs_beta": 1000000},     # bottom-up from the second step on
               {"bfs_alpha": 1000000, "bfs_beta": 1},           # alternate bottom-up and top-down
               {}]                                              # the default switch


@pytest.mark.parametrize("tuning", DO_VARIANTS)
def test_bfs_direction_optimizing(gpu, rmat14, tuning):
    """Bottom-up steps give the same levels as top-down ones, on a symmetric
    graph (wave and thread bottom-up kernels), a directed one (in-edges) and
    graphs with isolated and unreachable vertices."""
    g, _ = rmat14
    cases = [(g, [graphgen.max_degree_vertex(g)] + graphgen.sample_roots(g, 3, seed=11).tolist())]
    gd = graphgen.rmat(12, symmetrize=False)
    cases.append((gd, graphgen.sample_roots(gd, 3, seed=12).tolist()))
    gp = graphgen.from_edges(9, [0, 1, 2, 5, 6], [1, 2, 3, 6, 7], symmetrize=True)
    cases.append((gp, [0, 4, 5]))
    gs = graphgen.from_edges(3001, np.zeros(3000, dtype=int), np.arange(1, 3001), symmetrize=True)
    cases.append((gs, [0, 7]))
    for graph, roots in cases:
        P = load(gpu, graph, None, tuning)
        lev = gpu.bfs(P, roots).cpu().numpy()
        for i, r in enumerate(roots):
            assert np.array_equal(lev[i], oracle.bfs(graph.offsets, graph.cols, r)), (tuning, graph.n, r)


# ------------------------------------------------------------------ edges

def test_degenerate_graphs(gpu):
    # single vertex
    g = graphgen.from_edges(1, [], [], symmetrize=True)
    P = load(gpu, g, np.zeros(0, np.int32))
    assert gpu.bfs(P, [0]).cpu().numpy().tolist() == [[0]]
    assert gpu.sssp(P, [0]).cpu().numpy().tolist() == [[0]]
    assert np.allclose(gpu.pagerank(P, 0.85, 5).cpu().numpy(), [1.0])
    assert gpu.bc(P, [0]).cpu().numpy().tolist() == [0.0]
    # isolated root, disconnected pieces
    g = graphgen.from_edges(7, [0, 1, 4], [1, 2, 5], symmetrize=True)
    w = graphgen.weights(g)
    P = load(gpu, g, w)
    assert np.array_equal(gpu.bfs(P, [3]).cpu().numpy()[0], oracle.bfs(g.offsets, g.cols, 3))
    assert np.array_equal(gpu.bfs(P, [0]).cpu().numpy()[0], oracle.bfs(g.offsets, g.cols, 0))
    assert np.array_equal(gpu.sssp(P, [5]).cpu().numpy()[0], oracle.sssp(g.offsets, g.cols, w, 5))
    # zero iterations return r_0
    assert np.allclose(gpu.pagerank(P, 0.85, 0).cpu().numpy(), 1.0 / 7)


def test_star_hub_beyond_thresholds(gpu):
    n = 20000  # hub degree above the default hub threshold and many chunks
    g = graphgen.from_edges(n + 1, np.zeros(n, dtype=int), np.arange(1, n + 1), symmetrize=True)
    P = load(gpu, g, graphgen.weights(g))
    lev = gpu.bfs(P, [5]).cpu().numpy()[0]
    assert lev[0] == 1 and lev[5] == 0 and np.all(np.delete(lev, [0, 5]) == 2)
    r = gpu.pagerank(P, 0.85, 10).cpu().numpy()
    assert pr_rel_l1(r, oracle.pagerank(g.offsets, g.cols, 0.85, 10)) <= 1e-5
    b = gpu.bc(P, [0, 1, 2]).cpu().numpy()
    assert bc_close(b, oracle.bc(g.offsets, g.cols, [0, 1, 2]))


def test_long_path(gpu):
    n = 3000  # many levels with one-vertex frontiers
    g = graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n), symmetrize=True)
    w = graphgen.weights(g)
    P = load(gpu, g, w)
    assert np.array_equal(gpu.bfs(P, [17]).cpu().numpy()[0], np.abs(np.arange(n) - 17))
    assert np.array_equal(gpu.sssp(P, [0]).cpu().numpy()[0], oracle.sssp(g.offsets, g.cols, w, 0))
    b = gpu.bc(P, [0, n - 1]).cpu().numpy()
    assert bc_close(b, oracle.bc(g.offsets, g.cols, [0, n - 1]))


def test_sssp_overflow_reported(gpu):
    g = graphgen.from_edges(3, [0, 1], [1, 2], symmetrize=False)
    w = np.array([2**31 - 10, 2**31 - 10], dtype=np.int32)
    P = load(gpu, g, w)
    with pytest.raises(gpu.TGError) as ei:
        gpu.sssp(P, [0])
    assert ei.value.code == gpu.TG_ERANGE
    # a large edge that is not on the shortest path is fine
    g = graphgen.from_edges(3, [0, 0, 1], [1, 2, 2], symmetrize=False)
    w = np.array([1, 2**31 - 2, 1], dtype=np.int32)
    P = load(gpu, g, w)
    assert gpu.sssp(P, [0]).cpu().numpy().tolist() == [[0, 1, 2]]


def test_errors(gpu, rmat14):
    g, _ = rmat14
    P = load(gpu, g)
    with pytest.raises(gpu.TGError) as ei:
        gpu.sssp(P, [0])
    assert ei.value.code == gpu.TG_EUNSUPPORTED
    with pytest.raises(gpu.TGError) as ei:
        gpu.bfs(P, [g.n])
    assert ei.value.code == gpu.TG_EINVAL
    with pytest.raises(gpu.TGError):
        gpu.pagerank(P, 1.5, 3)


def test_determinism(gpu, rmat14):
    g, w = rmat14
    P = load(gpu, g, w)
    a = gpu.pagerank(P, 0.85, 10).cpu().numpy()
    b = gpu.pagerank(P, 0.85, 10).cpu().numpy()
    assert np.array_equal(a, b)
    s1 = gpu.sssp(P, [3]).cpu().numpy()
    s2 = gpu.sssp(P, [3]).cpu().numpy()
    assert np.array_equal(s1, s2)


def test_retune_keeps_results(gpu, rmat14):
    g, w = rmat14
    P = load(gpu, g, w)
    root = graphgen.max_degree_vertex(g)
    ref_lev = oracle.bfs(g.offsets, g.cols, root)
    ref_pr = oracle.pagerank(g.offsets, g.cols, 0.85, 10)
    for tuning in (SMALL_BINS, {"pr_lds_verts": 0, "bfs_lds_words": 0, "bfs_lds_min_vblocks": 0},
                   dict(SMALL_BINS, pr_xcd=0), {"pr_xcd": 0}, {"pr_rows": 512}, {"pr_rows": 256, "pr_xcd": 0},
                   None):
        gpu.partition_retune(P, tuning)
        assert np.array_equal(gpu.bfs(P, [root]).cpu().numpy()[0], ref_lev)
        assert pr_rel_l1(gpu.pagerank(P, 0.85, 10).cpu().numpy(), ref_pr) <= 1e-5
        assert np.array_equal(gpu.sssp(P, [root]).cpu().numpy()[0], oracle.sssp(g.offsets, g.cols, w, root))
    with pytest.raises(gpu.TGError):
        gpu.partition_retune(P, {"hub_min_deg": 10, "block_min_deg": 100})
