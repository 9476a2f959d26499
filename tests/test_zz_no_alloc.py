"""The allocation-free BFS entry point (bfs_noalloc, through the C ABI)
against bfs() and the oracle: two calls in a row on one GPU, the second on a
smaller graph (the shared scratch keeps the first call's contents), and its
error cases."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def call_noalloc(tg, part, roots, out):
    r = np.ascontiguousarray(np.asarray(roots, dtype=np.int32))
    return tg._load().bfs_noalloc(part.handle, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), r.size,
                                  out.data_ptr(), None)


def test_noalloc_matches_bfs_on_two_calls(gpu):
    import torch
    tg = gpu
    # first a larger graph (several bins, hub chunks, bottom-up steps), then
    # a smaller one: the second call must not see the first call's state
    for scale, nroots in ((14, 6), (10, 3)):
        g = graphgen.rmat(scale)
        G = tg.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True)
        P = tg.partition_by_degree(G)
        roots = [graphgen.max_degree_vertex(g)] + graphgen.sample_roots(g, nroots - 1, seed=scale).tolist()
        ref = tg.bfs(P, roots)
        out = torch.full((nroots, g.n), -7, dtype=torch.int32, device="cuda")
        assert call_noalloc(tg, P, roots, out) == 0, tg._load().tg_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), scale
        got = out.cpu().numpy()
        for i in (0, nroots - 1):
            assert np.array_equal(got[i], oracle.bfs(g.offsets, g.cols, roots[i])), (scale, roots[i])


def test_noalloc_directed_and_errors(gpu):
    import torch
    tg = gpu
    g = graphgen.rmat(12, symmetrize=False)
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, symmetric=False)
    P = tg.partition_by_degree(G)
    roots = graphgen.sample_roots(g, 4, seed=9).tolist()
    out = torch.empty((4, g.n), dtype=torch.int32, device="cuda")
    assert call_noalloc(tg, P, roots, out) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, tg.bfs(P, roots))
    # a root out of range, a hybrid partition
    assert call_noalloc(tg, P, [g.n], out) == tg.TG_EINVAL
    H = tg.partition_by_degree(G, "high", 0.3)
    assert call_noalloc(tg, H, roots, out) == tg.TG_EUNSUPPORTED
    # a partition larger than the scratch array: 9 M vertices need about 75 MB
    n = 9_000_000
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = 2
    off[1] = 1
    cols = np.array([1, 0], dtype=np.int32)
    B = tg.partition_by_degree(tg.graph_load_csr(n, off, cols, symmetric=True))
    big = torch.empty((1, n), dtype=torch.int32, device="cuda")
    assert call_noalloc(tg, B, [0], big) == tg.TG_ENOMEM
    assert b"scratch" in tg._load().tg_last_error()
