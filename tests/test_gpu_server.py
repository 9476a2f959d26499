"""Serving: queries admitted while others run (continuous batching) give the
same results as solo runs; admission by slots and memory; timeouts."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def graphs(gpu):
    out = []
    for g in (graphgen.rmat(12), graphgen.rmat(11, symmetrize=False), graphgen.uniform(3000, 9000, seed=5)):
        w = graphgen.weights(g, seed=7)
        G = gpu.graph_load_csr(g.n, g.offsets, g.cols, w, symmetric=g.symmetric)
        out.append((g, w, G, gpu.partition_by_degree(G)))
    return out


def expected(g, w, kind, root):
    return oracle.bfs(g.offsets, g.cols, root) if kind == 0 else oracle.sssp(g.offsets, g.cols, w, root)


def run_mix(gpu, graphs, server, n_queries, seed, waves=4):
    import torch
    rng = np.random.default_rng(seed)
    gids = [server.add_graph(P) for (_, _, _, P) in graphs]
    jobs = []
    pending = []
    for wave in range(waves):
        for _ in range(n_queries // waves):
            gi = int(rng.integers(len(graphs)))
            g, w, _, _ = graphs[gi]
            kind = int(rng.integers(2))
            root = int(rng.choice(graphgen.sample_roots(g, 50, seed=int(rng.integers(1 << 30)))))
            out = torch.empty(g.n, dtype=torch.int32, device="cuda")
            t = server.submit(gids[gi], kind, root, out)
            jobs.append((gi, kind, root, out, t))
            pending.append(t)
        # let part of the work finish before the next wave arrives
        for t in pending[: len(pending) // 2]:
            server.wait(t)
        pending = pending[len(pending) // 2:]
    for t in pending:
        server.wait(t)
    for gi, kind, root, out, _ in jobs:
        g, w, _, _ = graphs[gi]
        assert np.array_equal(out.cpu().numpy(), expected(g, w, kind, root)), (gi, kind, root)
    return server.stats()


def test_continuous_batching_results_match_solo(gpu, graphs):
    S = gpu.Server(max_slots=64)
    st = run_mix(gpu, graphs, S, 160, seed=1)
    assert st["completed"] == 160
    assert st["max_concurrent"] > 1
    S.close()


@pytest.mark.parametrize("max_slots", [64, 1])
def test_solo_sssp_lanes(gpu, graphs, max_slots):
    """SSSP queries served as single searches (sssp_solo_min_vertices = 0:
    every graph), beside BFS queries in the slot engines: every result
    equals the oracle; with max_slots 1 one query per (graph, kind) runs at
    a time."""
    S = gpu.Server(max_slots=max_slots, sssp_solo_min_vertices=0, sssp_solo_min_skew=0)
    st = run_mix(gpu, graphs, S, 96, seed=3)
    assert st["completed"] == 96
    if max_slots == 1:
        assert st["max_concurrent"] <= 2 * len(graphs)
    S.close()


def test_solo_rule_follows_degree_skew(gpu):
    """With no size floor, the default skew rule serves SSSP on a star (hub
    degree far above the mean) as single searches, which run no slot-engine
    supersteps, and on a ring (every degree 2) through the slot engine; both
    give the oracle's distances."""
    import torch
    n = 2000
    star = graphgen.from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n), symmetrize=True)
    ring = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n, symmetrize=True)
    for g, solo in ((star, True), (ring, False)):
        w = graphgen.weights(g, seed=6)
        P = gpu.partition_by_degree(gpu.graph_load_csr(g.n, g.offsets, g.cols, w))
        S = gpu.Server(sssp_solo_min_vertices=0)
        gid = S.add_graph(P)
        roots = [0, 1, n // 2, n - 1]
        outs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in roots]
        for t in [S.submit(gid, gpu.TG_QUERY_SSSP, r, o) for r, o in zip(roots, outs)]:
            S.wait(t)
        for r, o in zip(roots, outs):
            assert np.array_equal(o.cpu().numpy(), oracle.sssp(g.offsets, g.cols, w, r)), (solo, r)
        assert (S.stats()["supersteps"] == 0) == solo
        S.close()
    with pytest.raises(gpu.TGError) as ei:
        gpu.Server(sssp_solo_min_skew=-1)
    assert ei.value.code == gpu.TG_EINVAL


def test_solo_sssp_memory_cap(gpu, graphs):
    """A memory cap of one SSSP query admits solo searches one at a time."""
    import torch
    g, w, _, P = graphs[0]
    per_sssp = 4 * g.n + (2 * g.n + 7) // 8
    S = gpu.Server(memory_cap_bytes=per_sssp, sssp_solo_min_vertices=0, sssp_solo_min_skew=0)
    gid = S.add_graph(P)
    roots = graphgen.sample_roots(g, 10, seed=4)
    outs = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in roots]
    ts = [S.submit(gid, gpu.TG_QUERY_SSSP, int(r), o) for r, o in zip(roots, outs)]
    for t in ts:
        S.wait(t)
    for r, o in zip(roots, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.sssp(g.offsets, g.cols, w, int(r)))
    assert S.stats()["max_concurrent"] == 1
    S.close()


def test_one_at_a_time_mode(gpu, graphs):
    S = gpu.Server(max_slots=1)
    st = run_mix(gpu, graphs, S, 24, seed=2)
    assert st["completed"] == 24
    assert st["max_concurrent"] <= 2 * len(graphs)  # one per (graph, kind)
    S.close()


def test_memory_admission(gpu, graphs):
    import torch
    g, w, _, P = graphs[0]
    per_bfs = (3 * g.n + 7) // 8
    with pytest.raises(gpu.TGError) as ei:
        S = gpu.Server(memory_cap_bytes=per_bfs - 1)
        gid = S.add_graph(P)
        S.submit(gid, gpu.TG_QUERY_BFS, 0, torch.empty(g.n, dtype=torch.int32, device="cuda"))
    assert ei.value.code == gpu.TG_ENOMEM
    S.close()
    S = gpu.Server(memory_cap_bytes=2 * per_bfs)  # two BFS queries at a time
    gid = S.add_graph(P)
    roots = graphgen.sample_roots(g, 12, seed=9)
    outs = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in roots]
    ts = [S.submit(gid, gpu.TG_QUERY_BFS, int(r), o) for r, o in zip(roots, outs)]
    for t in ts:
        S.wait(t)
    for r, o in zip(roots, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.bfs(g.offsets, g.cols, int(r)))
    assert S.stats()["max_concurrent"] <= 2
    S.close()


def test_timeout_and_errors(gpu):
    import torch
    n = 6000  # a long path: thousands of supersteps
    g = graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n), symmetrize=True)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True)
    P = gpu.partition_by_degree(G)
    S = gpu.Server()
    gid = S.add_graph(P)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    t = S.submit(gid, gpu.TG_QUERY_BFS, 0, out)
    with pytest.raises(gpu.TGError) as ei:
        S.wait(t, timeout_us=0)
    assert ei.value.code == gpu.TG_ETIMEOUT
    S.wait(t)
    assert np.array_equal(out.cpu().numpy(), np.arange(n))
    with pytest.raises(gpu.TGError) as ei:
        S.submit(gid + 5, gpu.TG_QUERY_BFS, 0, out)
    assert ei.value.code == gpu.TG_EINVAL
    with pytest.raises(gpu.TGError) as ei:
        S.submit(gid, gpu.TG_QUERY_SSSP, 0, out)  # no weights
    assert ei.value.code == gpu.TG_EUNSUPPORTED
    with pytest.raises(gpu.TGError):
        S.submit(gid, gpu.TG_QUERY_BFS, n, out)
    S.close()


@pytest.mark.parametrize("solo", [None, 0])
def test_overflowing_query_does_not_poison_its_lane(gpu, solo):
    """An SSSP query whose distances do not fit in int32 fails with
    TG_ERANGE; queries before, beside and after it on the same (graph, SSSP)
    lane keep their exact results (the overflow verdict is per query), in
    the slot engine and with solo searches."""
    import torch
    big = 2**31 - 10
    # 0 -> 1 -> 2 with huge weights (root 0 overflows at vertex 2); a path
    # 3 -> 4 -> ... -> 202 with small weights keeps other queries in flight
    src = [0, 1] + list(range(3, 202))
    dst = [1, 2] + list(range(4, 203))
    g = graphgen.from_edges(203, np.array(src), np.array(dst), symmetrize=False)
    wmap = {(0, 1): big, (1, 2): big}
    w = np.array([wmap.get((u, int(v)), 3 + (u % 5)) for u in range(g.n)
                  for v in g.cols[g.offsets[u]:g.offsets[u + 1]]], dtype=np.int32)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, w)
    P = gpu.partition_by_degree(G)
    S = gpu.Server(sssp_solo_min_vertices=solo, sssp_solo_min_skew=solo)
    gid = S.add_graph(P)
    roots_before = [3, 1, 10]
    roots_after = [0, 3, 1, 50, 4, 0, 200, 1]
    outs, tickets = [], []
    for r in roots_before + [0] + roots_after:
        o = torch.empty(g.n, dtype=torch.int32, device="cuda")
        outs.append((r, o))
        tickets.append(S.submit(gid, gpu.TG_QUERY_SSSP, r, o))
    for (r, o), t in zip(outs, tickets):
        if r == 0:
            with pytest.raises(gpu.TGError) as ei:
                S.wait(t)
            assert ei.value.code == gpu.TG_ERANGE
        else:
            S.wait(t)
            assert np.array_equal(o.cpu().numpy(), oracle.sssp(g.offsets, g.cols, w, r)), r
    # the lane stays healthy for later queries
    o = torch.empty(g.n, dtype=torch.int32, device="cuda")
    S.wait(S.submit(gid, gpu.TG_QUERY_SSSP, 3, o))
    assert np.array_equal(o.cpu().numpy(), oracle.sssp(g.offsets, g.cols, w, 3))
    # every query, failed or not, gave its admitted bytes back
    assert S.stats()["memory_in_use"] == 0
    S.close()
    with pytest.raises(gpu.TGError) as ei:
        gpu.sssp(P, [0])
    assert ei.value.code == gpu.TG_ERANGE


def test_add_graph_while_queries_run(gpu, graphs):
    """Graphs registered while earlier queries are in flight (the worker walks
    its lanes meanwhile): every result, old and new, equals the oracle."""
    import torch
    n = 3000
    path = graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n), symmetrize=True)
    PG = gpu.graph_load_csr(path.n, path.offsets, path.cols, symmetric=True)
    PP = gpu.partition_by_degree(PG)
    S = gpu.Server()
    pid = S.add_graph(PP)
    long_out = torch.empty(n, dtype=torch.int32, device="cuda")
    long_t = S.submit(pid, gpu.TG_QUERY_BFS, 0, long_out)  # thousands of supersteps
    jobs = []
    for rep in range(4):  # grow the lane table several times over
        for (g, w, _, P) in graphs:
            gid = S.add_graph(P)
            for kind in (0, 1):
                root = int(graphgen.sample_roots(g, 3, seed=rep)[kind])
                out = torch.empty(g.n, dtype=torch.int32, device="cuda")
                jobs.append((g, w, kind, root, out, S.submit(gid, kind, root, out)))
    for (g, w, kind, root, out, t) in jobs:
        S.wait(t)
        assert np.array_equal(out.cpu().numpy(), expected(g, w, kind, root)), (kind, root)
    S.wait(long_t)
    assert np.array_equal(long_out.cpu().numpy(), np.arange(n))
    S.close()
