"""Pins for the oracle's SSSP and BFS (CPU only).

Each check compares the oracle with something other than itself: values worked
by hand, Floyd-Warshall written here, scipy's independent shortest-path
routines, and the optimality certificate (which is itself pinned by planted
mistakes that it must reject).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import fpp_inputs as fi
import oracle
from golden_io import INF, load_sp_fixture


def floyd_warshall(g, unit=False):
    n = g.num_vertices
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0.0)
    deg = g.out_degree()
    src = np.repeat(np.arange(n), deg)
    w = np.ones(g.num_edges) if (unit or g.weight is None) else g.weight.astype(np.float64)
    for s, t, ww in zip(src, g.col, w):
        if ww < D[s, t]:
            D[s, t] = ww
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    out = np.where(np.isinf(D), INF, D).astype(np.int64)
    return out.astype(np.int32)


def to_scipy(g, unit=False):
    n = g.num_vertices
    src = np.repeat(np.arange(n), g.out_degree())
    w = np.ones(g.num_edges) if (unit or g.weight is None) else g.weight.astype(np.float64)
    # duplicates: keep the minimum weight (coo->csr would sum them)
    key = src.astype(np.int64) * n + g.col
    order = np.lexsort((w, key))
    key, w = key[order], w[order]
    first = np.ones(key.size, bool)
    first[1:] = key[1:] != key[:-1]
    key, w = key[first], w[first]
    return sp.csr_matrix((w, (key // n, key % n)), shape=(n, n))


def test_hand_fixture():
    nv, edges, expect = load_sp_fixture("sssp_bfs_hand8.txt")
    s, d, w = zip(*edges)
    g = fi.from_edges(nv, s, d, w)
    for (kind, src), vec in expect.items():
        got = oracle.sssp(g, [src])[0] if kind == "sssp" else oracle.bfs(g, [src])[0]
        np.testing.assert_array_equal(got, vec, err_msg=f"{kind} from {src}")


@pytest.mark.parametrize("seed", range(12))
def test_dijkstra_vs_floyd_warshall(seed):
    n = [1, 2, 5, 17, 40, 64][seed % 6]
    g = fi.random_small(n, 3 * n, seed, wmax=[1, 9, 255][seed % 3])
    fw = floyd_warshall(g)
    got = oracle.sssp(g, np.arange(n))
    np.testing.assert_array_equal(got, fw)


@pytest.mark.parametrize("seed", range(6))
def test_bfs_vs_floyd_warshall_unit(seed):
    n = [3, 9, 33, 64, 50, 20][seed]
    g = fi.random_small(n, 2 * n, 100 + seed)
    fw = floyd_warshall(g, unit=True)
    np.testing.assert_array_equal(oracle.bfs(g, np.arange(n)), fw)
    # BFS is SSSP with unit weights
    gu = fi.Graph(g.num_vertices, g.row_ptr, g.col, np.ones(g.num_edges, np.uint32))
    np.testing.assert_array_equal(oracle.bfs(g, np.arange(n)), oracle.sssp(gu, np.arange(n)))


def test_dijkstra_vs_scipy_rmat12():
    g = fi.rmat(12, seed=1, weights=(1, 255), weight_seed=101)
    srcs = fi.sources_uniform(g, 16, 7)
    ref = csg.dijkstra(to_scipy(g), directed=True, indices=srcs)
    ref = np.where(np.isinf(ref), INF, ref).astype(np.int32)
    np.testing.assert_array_equal(oracle.sssp(g, srcs), ref)
    refb = csg.shortest_path(to_scipy(g, unit=True), method="D", directed=True, unweighted=True,
                             indices=srcs)
    refb = np.where(np.isinf(refb), INF, refb).astype(np.int32)
    np.testing.assert_array_equal(oracle.bfs(g, srcs), refb)


def test_grid_distances_closed_form():
    # unit-weight grid: BFS level = Manhattan distance
    g = fi.grid(7, 11, weights=None)
    lv = oracle.bfs(g, [0, 40])
    r, c = np.divmod(np.arange(77), 11)
    np.testing.assert_array_equal(lv[0], r + c)
    r0, c0 = divmod(40, 11)
    np.testing.assert_array_equal(lv[1], np.abs(r - r0) + np.abs(c - c0))


def test_certificate_accepts_exact_and_rejects_planted_mistakes():
    g = fi.rmat(10, seed=9, weights=(1, 50), weight_seed=19)
    srcs = fi.sources_uniform(g, 4, 3)
    D = oracle.sssp(g, srcs)
    L = oracle.bfs(g, srcs)
    rng = np.random.default_rng(0)
    for i, s in enumerate(srcs):
        assert oracle.sp_certificate(g, s, D[i]) == 0
        assert oracle.sp_certificate(g, s, L[i], unit_weights=True) == 0
        fin = np.flatnonzero((D[i] != INF) & (np.arange(g.num_vertices) != s))
        v = rng.choice(fin)
        for delta in (+1, -1):
            bad = D[i].copy()
            bad[v] += delta
            assert oracle.sp_certificate(g, s, bad) != 0
        bad = D[i].copy()
        bad[v] = INF
        assert oracle.sp_certificate(g, s, bad) != 0
        bad = D[i].copy()
        bad[s] = 1
        assert oracle.sp_certificate(g, s, bad) != 0
        unreach = np.flatnonzero(D[i] == INF)
        if unreach.size:
            bad = D[i].copy()
            bad[unreach[0]] = 10 ** 6
            assert oracle.sp_certificate(g, s, bad) != 0


def test_edge_cases():
    # single vertex, no edges
    g = fi.from_edges(1, [], [], [])
    assert oracle.sssp(g, [0])[0, 0] == 0
    assert oracle.bfs(g, [0])[0, 0] == 0
    # source without out-edges; self-loops only
    g = fi.from_edges(3, [1, 1], [1, 0], [5, 2])
    np.testing.assert_array_equal(oracle.sssp(g, [0])[0], [0, INF, INF])
    np.testing.assert_array_equal(oracle.sssp(g, [1])[0], [2, 0, INF])
    # long chain with maximum weight stays exact in int32
    n = 1000
    g = fi.from_edges(n, np.arange(n - 1), np.arange(1, n), np.full(n - 1, 2_000_000))
    d = oracle.sssp(g, [0])[0]
    np.testing.assert_array_equal(d, np.arange(n, dtype=np.int64) * 2_000_000)
