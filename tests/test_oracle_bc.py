"""Pins of the betweenness-centrality oracle (oracle/bc.py), CPU only.

- **Brandes vs brute force.** The two sweeps equal brute-force enumeration of
  every simple path on random tiny multigraphs (parallel edges, self-loops,
  weighted and unit).
- **Closed forms.** A path graph gives BC(v_i) = 2 i (n-1-i) over all
  sources; a star's centre gives k(k-1).
- **Hand example.** A diamond with parallel edges, worked out below.
"""
import numpy as np
import pytest

import fpp_inputs as fi
from oracle import bc


@pytest.mark.parametrize("seed", range(8))
def test_brandes_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 8))
    g = fi.random_small(n, int(rng.integers(n, 3 * n + 4)), 500 + seed, wmax=3)
    srcs = np.arange(n)
    for unit in (True, False):
        np.testing.assert_allclose(bc.dependencies(g, srcs, unit), bc.brute_force(g, srcs, unit),
                                   rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [2, 5, 9])
def test_path_graph_closed_form(n):
    s = list(range(n - 1)) + list(range(1, n))
    t = list(range(1, n)) + list(range(n - 1))
    g = fi.from_edges(n, s, t)
    got = bc.centrality(g, np.arange(n))
    i = np.arange(n)
    np.testing.assert_allclose(got, 2.0 * i * (n - 1 - i))


def test_star_closed_form():
    k = 6
    s = [0] * k + list(range(1, k + 1))
    t = list(range(1, k + 1)) + [0] * k
    g = fi.from_edges(k + 1, s, t, [3] * (2 * k))
    for unit in (True, False):
        got = bc.centrality(g, np.arange(k + 1), unit)
        assert got[0] == pytest.approx(k * (k - 1)) and np.all(got[1:] == 0)


def test_diamond_with_parallel_edges_by_hand():
    # 0->1 (twice), 0->2, 1->3, 2->3, all weight 1.  From source 0: sigma(1) = 2,
    # sigma(2) = 1, sigma(3) = 3; delta(1) = 2/3 (paths to 3 through 1),
    # delta(2) = 1/3, delta(3) = 0.
    g = fi.from_edges(4, [0, 0, 0, 1, 2], [1, 1, 2, 3, 3], [1, 1, 1, 1, 1])
    d = bc.dependencies(g, [0], unit=False)[0]
    np.testing.assert_allclose(d, [0.0, 2.0 / 3.0, 1.0 / 3.0, 0.0])
    # a heavier parallel edge is not a shortest path
    g2 = fi.from_edges(4, [0, 0, 0, 1, 2], [1, 1, 2, 3, 3], [1, 5, 1, 1, 1])
    np.testing.assert_allclose(bc.dependencies(g2, [0], unit=False)[0], [0.0, 0.5, 0.5, 0.0])
    np.testing.assert_allclose(bc.dependencies(g2, [0], unit=True)[0], [0.0, 2.0 / 3.0, 1.0 / 3.0, 0.0])


@pytest.mark.parametrize("seed", range(4))
def test_dependencies_sum_to_interior_vertices(seed):
    """With unit weights every shortest s-t path has d(s, t) - 1 interior
    vertices, so a source's dependencies sum to the sum over reached t of
    d(s, t) - 1 (levels from the oracle's BFS)."""
    import oracle
    g = fi.rmat(8, seed=600 + seed)
    srcs = fi.sources_uniform(g, 5, 700 + seed)
    dep = bc.dependencies(g, srcs, unit=True)
    lv = oracle.bfs(g, srcs).astype(np.int64)
    for i in range(len(srcs)):
        reached = lv[i][(lv[i] > 0) & (lv[i] != 0x7FFFFFFF)]
        assert dep[i].sum() == pytest.approx(float(np.sum(reached - 1)), rel=1e-12)
