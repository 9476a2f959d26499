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
