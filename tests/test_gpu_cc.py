"""GPU connected components against the oracle: labels are the smallest
original id of each component, compared element by element (bit-exact)."""
import numpy as np
import pytest

import graphgen
import oracle
pytestmark = pytest.mark.gpu

# small degree thresholds: every bin and multi-chunk hubs on small graphs
SMALL_BINS = {"hub_min_deg": 300, "block_min_deg": 100, "wave_min_deg": 24, "g16_min_deg": 6,
              "g4_min_deg": 2, "hub_chunk": 256}


def load(tg, g, weights=None, tuning=None):
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, weights, symmetric=g.symmetric)
    return tg.partition_by_degree(G, tuning=tuning)


@pytest.mark.parametrize("tuning", [None, SMALL_BINS])
def test_cc_rmat(gpu, tuning):
    for g in (graphgen.rmat(14), graphgen.rmat(12, symmetrize=False), graphgen.rmat(12, seed=9, permute=False)):
        P = load(gpu, g, None, tuning)
        lab = gpu.cc(P).cpu().numpy()
        assert np.array_equal(lab, oracle.cc(g.offsets, g.cols)), (tuning, g.n, g.symmetric)


def test_cc_many_components(gpu):
    # sparse uniform graphs: thousands of small components and isolated vertices
    for sym in (True, False):
        rng = np.random.default_rng(5)
        n, m = 20000, 9000
        g = graphgen.from_edges(n, rng.integers(0, n, m), rng.integers(0, n, m), symmetrize=sym)
        P = load(gpu, g)
        assert np.array_equal(gpu.cc(P).cpu().numpy(), oracle.cc(g.offsets, g.cols))


def test_cc_shapes(gpu):
    n = 20000  # star: one hub beyond every degree threshold
    star = graphgen.from_edges(n + 1, np.full(n, 7), np.delete(np.arange(n + 1), 7), symmetrize=True)
    path = graphgen.from_edges(3000, np.arange(2999), np.arange(1, 3000), symmetrize=True)  # long diameter
    single = graphgen.from_edges(1, [], [], symmetrize=True)
    empty = graphgen.from_edges(5, [], [], symmetrize=False)
    chain_dir = graphgen.from_edges(6, [5, 4, 3, 2, 1], [4, 3, 2, 1, 0], symmetrize=False)
    for g in (star, path, single, empty, chain_dir):
        P = load(gpu, g)
        assert np.array_equal(gpu.cc(P).cpu().numpy(), oracle.cc(g.offsets, g.cols)), g.n


def test_cc_hybrid_unsupported(gpu):
    g = graphgen.rmat(10)
    G = gpu.graph_load_csr(g.n, g.offsets, g.cols, symmetric=True)
    P = gpu.partition_by_degree(G, "high", 0.3)
    with pytest.raises(gpu.TGError):
        gpu.cc(P)
