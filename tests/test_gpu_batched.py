"""Batched (64-slot bitmask) BFS and SSSP: every root's result equals its
single-source run and the oracle (bit-exact)."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

SMALL_BINS = {"hub_min_deg": 300, "block_min_deg": 100, "wave_min_deg": 24, "g16_min_deg": 6,
              "g4_min_deg": 2, "hub_chunk": 256}


@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("tuning", [None, SMALL_BINS])
def test_batched_equals_oracle(gpu, sym, tuning):
    g = graphgen.rmat(12, symmetrize=sym)
    w = graphgen.weights(g, seed=8)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, w, symmetric=sym)
    P = gpu.partition_by_degree(G, tuning=tuning)
    # 70 roots: one full chunk of 64 and a ragged one; a repeated root; an isolated one
    roots = graphgen.sample_roots(g, 68, seed=2).tolist()
    roots += [roots[3], int(np.argmin(np.diff(g.offsets)))]
    lev = gpu.bfs_batched(P, roots).cpu().numpy()
    dist = gpu.sssp_batched(P, roots).cpu().numpy()
    single = gpu.bfs(P, roots[:5]).cpu().numpy()
    assert np.array_equal(single, lev[:5])
    for i, r in enumerate(roots):
        assert np.array_equal(lev[i], oracle.bfs(g.offsets, g.cols, r)), (i, r)
        assert np.array_equal(dist[i], oracle.sssp(g.offsets, g.cols, w, r)), (i, r)
    # reuse of the engine after a run gives the same answers
    lev2 = gpu.bfs_batched(P, roots[:7]).cpu().numpy()
    assert np.array_equal(lev2, lev[:7])


def test_batched_overflow_falls_back_exactly(gpu):
    g = graphgen.from_edges(4, [0, 1, 0], [1, 2, 3], symmetrize=False)
    # CSR edge order: (0,1), (0,3), (1,2)
    assert g.cols.tolist() == [1, 3, 2]
    w = np.array([2**31 - 10, 5, 2**31 - 10], dtype=np.int32)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, w)
    P = gpu.partition_by_degree(G)
    with pytest.raises(gpu.TGError) as ei:
        gpu.sssp_batched(P, [0])
    assert ei.value.code == gpu.TG_ERANGE
    assert gpu.sssp_batched(P, [3, 2, 1]).cpu().numpy().tolist() == [
        [2**31 - 1] * 3 + [0], [2**31 - 1, 2**31 - 1, 0, 2**31 - 1], [2**31 - 1, 0, 2**31 - 10, 2**31 - 1]]


@pytest.mark.parametrize("sym", [True, False])
def test_bc_batched_equals_oracle(gpu, sym):
    g = graphgen.rmat(11, symmetrize=sym)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, symmetric=sym)
    P = gpu.partition_by_degree(G, tuning=SMALL_BINS)
    srcs = graphgen.sample_roots(g, 70, seed=12).tolist() + [5, 5]
    got = gpu.bc_batched(P, srcs).cpu().numpy().astype(np.float64)
    ref = oracle.bc(g.offsets, g.cols, srcs)
    tol = 1e-4 * np.abs(ref) + 1e-6 * max(np.abs(ref).max(), 1.0)
    assert np.all(np.abs(got - ref) <= tol)
    single = gpu.bc(P, srcs[:3]).cpu().numpy().astype(np.float64)
    ref3 = oracle.bc(g.offsets, g.cols, srcs[:3])
    assert np.all(np.abs(single - ref3) <= 1e-4 * np.abs(ref3) + 1e-6 * max(ref3.max(), 1.0))


def test_bc_batched_many_graphs_in_one_chain(gpu):
    """Uneven graphs as one disjoint union: each graph's scores equal its solo run."""
    parts = [graphgen.rmat(s, seed=100 + i) for i, s in enumerate((7, 9, 8, 10, 7))]
    offs, cols, base = [np.zeros(1, dtype=np.int64)], [], 0
    edge_base = 0
    for g in parts:
        offs.append(g.offsets[1:] + edge_base)
        cols.append(g.cols + base)
        base += g.n
        edge_base += g.nnz
    U_off, U_col = np.concatenate(offs), np.concatenate(cols)
    G = gpu.graph_load_csr(base, U_off, U_col, symmetric=True)
    P = gpu.partition_by_degree(G)
    srcs, vbase = [], 0
    for g in parts:
        srcs += (graphgen.sample_roots(g, 6, seed=1) + vbase).tolist()
        vbase += g.n
    got = gpu.bc_batched(P, srcs).cpu().numpy().astype(np.float64)
    vbase = 0
    for g in parts:
        mine = [s - vbase for s in srcs if vbase <= s < vbase + g.n]
        ref = oracle.bc(g.offsets, g.cols, mine)
        sub = got[vbase:vbase + g.n]
        assert np.all(np.abs(sub - ref) <= 1e-4 * np.abs(ref) + 1e-6 * max(ref.max(), 1.0))
        vbase += g.n


def test_bc_multi_equals_each_graph(gpu):
    """bc_multi over graphs of uneven size (more graphs than worker streams,
    one directed, one with no sources): each graph's scores equal the oracle
    and its own bc_batched run."""
    specs = [(7, True), (10, True), (8, False), (12, True), (7, True), (9, True), (11, False), (8, True),
             (9, True), (6, True)]
    graphs, parts, srcs = [], [], []
    for i, (scale, sym) in enumerate(specs):
        g = graphgen.rmat(scale, seed=200 + i, symmetrize=sym)
        G = gpu.graph_load_csr(g.n, g.offsets, g.cols, symmetric=sym)
        graphs.append(g)
        parts.append(gpu.partition_by_degree(G, tuning=SMALL_BINS if i % 2 else None))
        srcs.append([] if i == 4 else graphgen.sample_roots(g, 40 + 13 * i, seed=i).tolist())
    got = gpu.bc_multi(parts, srcs)
    assert gpu.tg_last_stats()["graphs"] == len(specs)
    for i, g in enumerate(graphs):
        v = got[i].cpu().numpy().astype(np.float64)
        ref = oracle.bc(g.offsets, g.cols, srcs[i])
        assert np.all(np.abs(v - ref) <= 1e-4 * np.abs(ref) + 1e-6 * max(np.abs(ref).max(), 1.0)), i
        if srcs[i]:
            assert np.array_equal(v, gpu.bc_batched(parts[i], srcs[i]).cpu().numpy()), i
    with pytest.raises(gpu.TGError) as ei:
        gpu.bc_multi([parts[0], parts[0]], [srcs[0], srcs[0]])
    assert ei.value.code == gpu.TG_EINVAL
    with pytest.raises(gpu.TGError) as ei:
        gpu.bc_multi([parts[1], parts[0]], [srcs[1], [graphs[0].n]])
    assert ei.value.code == gpu.TG_EINVAL
    assert gpu.bc_multi([], []) == []


def test_tuning_cache_resolved_by_the_library(gpu, tmp_path, monkeypatch):
    """partition_by_degree(tuning_json=NULL) takes the cached entry keyed by
    device architecture and graph signature; "{}" and an unmatched graph
    take the built-in values."""
    import json
    import math
    g = graphgen.rmat(12)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True)
    avg = g.nnz / g.n
    key = f"gfx950:V2^{round(math.log2(g.n))}:deg{round(avg)}:sym"
    cfg = dict(SMALL_BINS, hub_chunk=512, bfs_alpha=7)
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({"gfx950:V2^30:deg1:dir": {"config": {"hub_chunk": 8192}},
                                key: {"config": cfg, "final_ms": {"all": 1.0}}}))
    monkeypatch.setenv("TG_TUNING_CACHE", str(path))
    P = gpu.partition_by_degree(G)
    info = P.info()
    assert info["tuning_source"] == "cache " + key
    for k, v in cfg.items():
        assert info["tuning"][k] == v, k
    root = graphgen.max_degree_vertex(g)
    assert np.array_equal(gpu.bfs(P, [root]).cpu().numpy()[0], oracle.bfs(g.offsets, g.cols, root))
    assert gpu.partition_by_degree(G, tuning="{}").info()["tuning_source"] == "caller"
    assert gpu.partition_by_degree(G, tuning="{}").info()["tuning"]["hub_chunk"] == 4096
    d = graphgen.rmat(12, symmetrize=False)
    D = gpu.graph_load_csr(d.n, d.offsets, d.cols, symmetric=False)
    assert gpu.partition_by_degree(D).info()["tuning_source"] == "built-in"
