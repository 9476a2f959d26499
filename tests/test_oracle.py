"""Pins for the oracle: each check ties it to something other than itself —
hand-worked values, closed forms, invariants, brute force on tiny inputs, or a
textbook routine from scipy / networkx."""
import itertools
import json
import os
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF = oracle.INF


def six():
    with open(os.path.join(GOLD, "six_vertex.json")) as f:
        return json.load(f)


def six_graph():
    g = six()
    e = np.array(g["undirected_edges"])
    csr = graphgen.from_edges(6, e[:, 0], e[:, 1], symmetrize=True)
    # weights: one per unordered pair, looked up from the edge list
    wmap = {}
    for a, b, w in g["undirected_edges"]:
        wmap[(a, b)] = wmap[(b, a)] = w
    w = np.array([wmap[(u, int(v))] for u in range(6)
                  for v in csr.cols[csr.offsets[u]:csr.offsets[u + 1]]], dtype=np.int32)
    return csr, w


def random_graph(n, m, seed, symmetrize):
    rng = np.random.default_rng(seed)
    return graphgen.from_edges(n, rng.integers(0, n, m), rng.integers(0, n, m),
                               symmetrize=symmetrize)


def to_nx(g, w=None):
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for k in range(g.offsets[u], g.offsets[u + 1]):
            if w is None:
                G.add_edge(u, int(g.cols[k]))
            else:
                G.add_edge(u, int(g.cols[k]), weight=int(w[k]))
    return G


def to_scipy(g, w=None):
    data = np.ones(g.nnz) if w is None else w.astype(np.float64)
    return sp.csr_matrix((data, g.cols, g.offsets), shape=(g.n, g.n))


# ----------------------------------------------------------------- BFS pins

def test_bfs_hand_worked():
    g, _ = six_graph()
    assert oracle.bfs(g.offsets, g.cols, 0).tolist() == six()["bfs_from_0"]


@pytest.mark.parametrize("n,root", [(1, 0), (7, 0), (7, 3), (50, 17)])
def test_bfs_path_closed_form(n, root):
    g = graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n), symmetrize=True)
    lev = oracle.bfs(g.offsets, g.cols, root)
    assert lev.tolist() == [abs(i - root) for i in range(n)]


@pytest.mark.parametrize("seed,sym", [(1, True), (2, False), (3, True), (4, False)])
def test_bfs_vs_scipy_and_networkx(seed, sym):
    g = random_graph(60, 90, seed, sym)
    ref = csg.shortest_path(to_scipy(g), unweighted=True, directed=True, indices=[5])[0]
    lev = oracle.bfs(g.offsets, g.cols, 5)
    expect = np.where(np.isinf(ref), INF, ref).astype(np.int64)
    assert np.array_equal(lev.astype(np.int64), expect)
    nxd = nx.single_source_shortest_path_length(to_nx(g), 5)
    for v in range(g.n):
        assert lev[v] == nxd.get(v, INF)


def test_bfs_parents_valid():
    g = graphgen.rmat(10, seed=7)
    root = graphgen.max_degree_vertex(g)
    lev, par = oracle.bfs(g.offsets, g.cols, root, parents=True)
    assert par[root] == root
    for v in range(g.n):
        if v == root:
            continue
        if lev[v] == INF:
            assert par[v] == -1
            continue
        p = par[v]
        assert lev[p] == lev[v] - 1
        assert v in g.cols[g.offsets[p]:g.offsets[p + 1]]
    # every edge changes the level by at most one along its direction
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    reach = lev[src] != INF
    assert np.all(lev[g.cols[reach]] <= lev[src[reach]] + 1)


def test_bfs_isolated_root_and_unreachable():
    g = graphgen.from_edges(5, [0, 1], [1, 2], symmetrize=False)
    assert oracle.bfs(g.offsets, g.cols, 4).tolist() == [INF, INF, INF, INF, 0]
    assert oracle.bfs(g.offsets, g.cols, 0).tolist() == [0, 1, 2, INF, INF]
    with pytest.raises(oracle.OracleError):
        oracle.bfs(g.offsets, g.cols, 5)


# ---------------------------------------------------------------- SSSP pins

def test_sssp_hand_worked():
    g, w = six_graph()
    assert oracle.sssp(g.offsets, g.cols, w, 0).tolist() == six()["sssp_from_0"]
    assert oracle.sssp(g.offsets, g.cols, w, 3).tolist() == six()["sssp_from_3"]


@pytest.mark.parametrize("seed,sym", [(11, False), (12, True), (13, False)])
def test_sssp_vs_floyd_warshall(seed, sym):
    g = random_graph(40, 120, seed, sym)
    w = graphgen.weights(g, seed=seed)
    fw = csg.floyd_warshall(to_scipy(g, w), directed=True)
    for root in (0, 7, 31):
        d = oracle.sssp(g.offsets, g.cols, w, root)
        ref = np.where(np.isinf(fw[root]), INF, fw[root]).astype(np.int64)
        assert np.array_equal(d.astype(np.int64), ref)
        bf = oracle.sssp(g.offsets, g.cols, w, root, method="bellman_ford")
        assert np.array_equal(bf, d)


def test_sssp_vs_networkx_dijkstra():
    g = graphgen.rmat(9, seed=5, symmetrize=False)
    w = graphgen.weights(g, seed=9)
    root = graphgen.max_degree_vertex(g)
    d = oracle.sssp(g.offsets, g.cols, w, root)
    ref = nx.single_source_dijkstra_path_length(to_nx(g, w), root)
    for v in range(g.n):
        assert d[v] == ref.get(v, INF)


def test_sssp_unit_weights_equal_bfs():
    g = graphgen.rmat(10, seed=3)
    w = np.ones(g.nnz, dtype=np.int32)
    for root in graphgen.sample_roots(g, 4, seed=1):
        assert np.array_equal(oracle.sssp(g.offsets, g.cols, w, root),
                              oracle.bfs(g.offsets, g.cols, root))


def test_sssp_triangle_and_tight_edges():
    g = graphgen.rmat(10, seed=4)
    w = graphgen.weights(g, seed=4)
    root = graphgen.max_degree_vertex(g)
    d = oracle.sssp64(g.offsets, g.cols, w, root)
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    big = np.iinfo(np.int64).max
    ok = d[src] != big
    assert np.all(d[g.cols[ok]] <= d[src[ok]] + w[ok])
    tight = np.zeros(g.n, dtype=bool)
    tight[g.cols[ok][d[g.cols[ok]] == d[src[ok]] + w[ok]]] = True
    reached = d != big
    reached[root] = False
    assert np.all(tight[reached])


def test_sssp_overflow_is_reported():
    g = graphgen.from_edges(3, [0, 1], [1, 2], symmetrize=False)
    w = np.array([2**31 - 10, 2**31 - 10], dtype=np.int32)
    with pytest.raises(oracle.DistanceOverflow):
        oracle.sssp(g.offsets, g.cols, w, 0)
    assert oracle.sssp64(g.offsets, g.cols, w, 0).tolist() == [0, 2**31 - 10, 2 * (2**31 - 10)]


# ------------------------------------------------------------ PageRank pins

def test_pagerank_hand_worked_first_step():
    g, _ = six_graph()
    r1 = oracle.pagerank(g.offsets, g.cols, 0.85, 1)
    exact = [float(Fraction(a, b)) for a, b in six()["pagerank_r1_fraction"]]
    assert np.allclose(r1, exact, rtol=0, atol=1e-15)
    e = np.array(six()["directed_edges"])
    gd = graphgen.from_edges(6, e[:, 0], e[:, 1], symmetrize=False)
    r1d = oracle.pagerank(gd.offsets, gd.cols, 0.85, 1, "uniform")
    exact = [float(Fraction(a, b)) for a, b in six()["directed_pagerank_r1_uniform_fraction"]]
    assert np.allclose(r1d, exact, rtol=0, atol=1e-15)


def google_matrix(g, d, dangling="uniform"):
    """Dense column-stochastic Google matrix built from the adjacency."""
    n = g.n
    A = np.zeros((n, n))
    deg = np.diff(g.offsets)
    for u in range(n):
        for v in g.cols[g.offsets[u]:g.offsets[u + 1]]:
            A[v, u] += 1.0 / deg[u]
        if deg[u] == 0 and dangling == "uniform":
            A[:, u] = 1.0 / n
    return d * A + (1 - d) / n * np.ones((n, n))


@pytest.mark.parametrize("seed,sym,k", [(21, True, 10), (22, False, 20), (23, False, 3)])
def test_pagerank_matches_matrix_power(seed, sym, k):
    g = random_graph(30, 45, seed, sym)  # sparse: has dangling vertices when directed
    G = google_matrix(g, 0.85)
    r = np.full(g.n, 1.0 / g.n)
    for _ in range(k):
        r = G @ r
    got = oracle.pagerank(g.offsets, g.cols, 0.85, k)
    assert np.allclose(got, r, rtol=1e-13, atol=1e-15)
    assert abs(got.sum() - 1.0) < 1e-12


def test_pagerank_drop_mode_matches_matrix_power():
    g = random_graph(30, 40, 31, False)
    deg = np.diff(g.offsets)
    assert (deg == 0).any()
    n = g.n
    A = np.zeros((n, n))
    for u in range(n):
        for v in g.cols[g.offsets[u]:g.offsets[u + 1]]:
            A[v, u] += 1.0 / deg[u]
    r = np.full(n, 1.0 / n)
    for _ in range(5):
        r = 0.85 * A @ r + 0.15 / n
    got = oracle.pagerank(g.offsets, g.cols, 0.85, 5, "drop")
    assert np.allclose(got, r, rtol=1e-13, atol=1e-15)
    assert got.sum() < 1.0


def test_pagerank_fixed_point_vs_networkx_and_eigen():
    g = random_graph(40, 70, 41, False)
    r = oracle.pagerank(g.offsets, g.cols, 0.85, 400)
    ref = nx.pagerank(to_nx(g), alpha=0.85, tol=1e-15, max_iter=100000)
    assert np.allclose(r, [ref[v] for v in range(g.n)], rtol=0, atol=1e-12)
    w, V = np.linalg.eig(google_matrix(g, 0.85))
    vec = np.real(V[:, np.argmax(np.real(w))])
    vec = vec / vec.sum()
    assert np.allclose(r, vec, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [3, 10])
def test_pagerank_star_closed_form(n):
    g = graphgen.from_edges(n + 1, np.zeros(n, dtype=int), np.arange(1, n + 1), symmetrize=True)
    d = 0.85
    r = oracle.pagerank(g.offsets, g.cols, d, 300)
    rc = (1 + d * n) / ((n + 1) * (1 + d))
    rl = (1 - d) / (n + 1) + d * rc / n
    assert abs(r[0] - rc) < 1e-13
    assert np.allclose(r[1:], rl, atol=1e-13)


def test_pagerank_regular_graph_is_uniform():
    n = 12
    g = graphgen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n, symmetrize=True)
    for k in (1, 5, 17):
        r = oracle.pagerank(g.offsets, g.cols, 0.85, k)
        assert np.allclose(r, 1.0 / n, rtol=0, atol=1e-16)


def test_pagerank_invariants_rmat():
    g = graphgen.rmat(11, seed=2)
    r = oracle.pagerank(g.offsets, g.cols, 0.85, 10)
    assert abs(r.sum() - 1.0) < 1e-12
    assert r.min() >= 0.15 / g.n - 1e-18


# ------------------------------------------------------------------ BC pins

def brute_force_bc(g, sources):
    """Enumerate every shortest path explicitly (tiny graphs only)."""
    n = g.n
    adj = [list(g.cols[g.offsets[u]:g.offsets[u + 1]]) for u in range(n)]
    out = [Fraction(0)] * n
    for s in sources:
        # all shortest paths from s, by growing paths level by level
        paths = {s: [[s]]}
        frontier = [s]
        seen = {s}
        while frontier:
            nxt = {}
            for u in frontier:
                for v in adj[u]:
                    if v in seen:
                        continue
                    nxt.setdefault(v, []).extend(p + [v] for p in paths[u])
            for v, ps in nxt.items():
                paths[v] = ps
                seen.add(v)
            frontier = list(nxt)
        for t, ps in paths.items():
            if t == s:
                continue
            for v in range(n):
                if v in (s, t):
                    continue
                through = sum(1 for p in ps if v in p[1:-1])
                out[v] += Fraction(through, len(ps))
    return [float(x) for x in out]


def test_bc_hand_worked():
    g, _ = six_graph()
    got, sig = oracle.bc(g.offsets, g.cols, [0], return_sigma=True)
    assert got.tolist() == six()["bc_source_0"]
    assert sig.tolist() == six()["sigma_source_0"]
    assert oracle.bc(g.offsets, g.cols, range(6)).tolist() == six()["bc_all_sources"]


@pytest.mark.parametrize("seed,sym", [(51, True), (52, False), (53, True)])
def test_bc_brute_force(seed, sym):
    g = random_graph(12, 22, seed, sym)
    srcs = list(range(g.n))
    assert np.allclose(oracle.bc(g.offsets, g.cols, srcs), brute_force_bc(g, srcs),
                       rtol=1e-12, atol=1e-12)
    sub = [1, 4, 9]
    assert np.allclose(oracle.bc(g.offsets, g.cols, sub), brute_force_bc(g, sub),
                       rtol=1e-12, atol=1e-12)


def test_bc_vs_networkx():
    g = graphgen.rmat(8, seed=6)
    ref = nx.betweenness_centrality(nx.Graph(to_nx(g)), normalized=False)
    got = oracle.bc(g.offsets, g.cols, range(g.n))
    assert np.allclose(got, [2 * ref[v] for v in range(g.n)], rtol=1e-10, atol=1e-9)
    gd = graphgen.rmat(8, seed=6, symmetrize=False)
    ref = nx.betweenness_centrality(to_nx(gd), normalized=False)
    got = oracle.bc(gd.offsets, gd.cols, range(gd.n))
    assert np.allclose(got, [ref[v] for v in range(gd.n)], rtol=1e-10, atol=1e-9)


def test_bc_closed_forms():
    n = 6  # star with n leaves
    g = graphgen.from_edges(n + 1, np.zeros(n, dtype=int), np.arange(1, n + 1), symmetrize=True)
    got = oracle.bc(g.offsets, g.cols, range(n + 1))
    assert got[0] == n * (n - 1) and np.all(got[1:] == 0)
    n = 9  # path
    g = graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n), symmetrize=True)
    got = oracle.bc(g.offsets, g.cols, range(n))
    assert got.tolist() == [2 * i * (n - 1 - i) for i in range(n)]
    n = 7  # complete graph
    s, d = zip(*itertools.combinations(range(n), 2))
    g = graphgen.from_edges(n, s, d, symmetrize=True)
    assert np.all(oracle.bc(g.offsets, g.cols, range(n)) == 0)


def test_bc_sum_equals_interior_count():
    g = graphgen.rmat(9, seed=8)
    srcs = graphgen.sample_roots(g, 10, seed=2)
    got = oracle.bc(g.offsets, g.cols, srcs)
    total = 0
    for s in srcs:
        lev = oracle.bfs(g.offsets, g.cols, s)
        fin = lev[lev != INF]
        total += int(np.sum(fin[fin > 0] - 1))
    assert abs(got.sum() - total) < 1e-6 * max(total, 1)


# ----------------------------------------------------------------- CC pins


def test_cc_hand_worked():
    # components {0, 1, 2}, {3, 4}, {5}, {6, 7} (edge 7 -> 6 directed: weak)
    g = graphgen.from_edges(8, [1, 2, 4, 7], [0, 1, 3, 6], symmetrize=False)
    assert oracle.cc(g.offsets, g.cols).tolist() == [0, 0, 0, 3, 3, 5, 6, 6]


def _components_brute(g):
    # undirected reachability by repeated relaxation of an adjacency matrix
    a = np.zeros((g.n, g.n), dtype=bool)
    for u in range(g.n):
        for v in g.cols[g.offsets[u]:g.offsets[u + 1]]:
            a[u, v] = a[v, u] = True
    reach = a | np.eye(g.n, dtype=bool)
    while True:
        nxt = reach | ((reach.astype(np.int32) @ reach.astype(np.int32)) > 0)
        if np.array_equal(nxt, reach):
            break
        reach = nxt
    return np.array([np.flatnonzero(reach[v]).min() for v in range(g.n)], dtype=np.int32)


@pytest.mark.parametrize("seed,sym", [(1, True), (2, False), (3, True), (4, False)])
def test_cc_brute_force(seed, sym):
    g = random_graph(40, 30, seed, sym)  # sparse: many components
    assert np.array_equal(oracle.cc(g.offsets, g.cols), _components_brute(g))


@pytest.mark.parametrize("seed,sym", [(5, True), (6, False)])
def test_cc_vs_scipy(seed, sym):
    g = random_graph(500, 420, seed, sym)
    k, comp = csg.connected_components(to_scipy(g), directed=True, connection="weak")
    lab = oracle.cc(g.offsets, g.cols)
    assert len(np.unique(lab)) == k
    # same partition, and the label is the smallest member
    for c in range(k):
        members = np.flatnonzero(comp == c)
        assert np.all(lab[members] == members.min())


def test_cc_invariants_rmat():
    g = graphgen.rmat(12, symmetrize=False, seed=3)
    lab = oracle.cc(g.offsets, g.cols)
    v = np.arange(g.n)
    assert np.all(lab <= v) and np.array_equal(lab[lab], lab)
    src = np.repeat(v, np.diff(g.offsets))
    assert np.array_equal(lab[src], lab[g.cols])  # every edge inside one component
    iso = np.diff(g.offsets) == 0
    indeg = np.bincount(g.cols, minlength=g.n)
    alone = iso & (indeg == 0)
    assert np.array_equal(lab[alone], v[alone])


def test_cc_empty_and_single():
    g = graphgen.from_edges(1, [], [], symmetrize=True)
    assert oracle.cc(g.offsets, g.cols).tolist() == [0]
    g = graphgen.from_edges(4, [], [], symmetrize=True)
    assert oracle.cc(g.offsets, g.cols).tolist() == [0, 1, 2, 3]
