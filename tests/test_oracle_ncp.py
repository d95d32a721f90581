"""Pins of the sweep-cut / NCP oracle (oracle/ncp.py), CPU only.

- **Incremental vs direct.** The incremental profile must equal the direct
  evaluation of the definition on random multigraphs.
- **Hand example.** A 4-cycle traversed in both directions, worked out by
  hand below.
- **Closed form.** Two cliques joined by one bridge: the best sweep cut is
  the seed's clique, with conductance 1 / (m(m-1) + 1).
- **Tie order and truncation.**
- **NCP.** Per-size-range minima.
"""
import numpy as np
import pytest

import fpp_inputs as fi
from oracle import ncp


def test_hand_worked_four_cycle():
    # 0-1-2-3-0, both directions: 8 directed edges, d(v) = 4, total volume 16.
    # p = 0.4, 0.3, 0.2, 0.1 sweeps 0, 1, 2, 3:
    #   {0}:       cut 4 (0-1, 0-3, each way), vol 4,  phi 4/4  = 1
    #   {0,1}:     cut 4 (1-2, 3-0),           vol 8,  phi 4/8  = 0.5
    #   {0,1,2}:   cut 4 (2-3, 3-0),           vol 12, phi 4/min(12,4) = 1
    #   {0,1,2,3}: cut 0,                      vol 16, undefined
    s = [0, 1, 1, 2, 2, 3, 3, 0]
    t = [1, 0, 2, 1, 3, 2, 0, 3]
    g = fi.from_edges(4, s, t)
    for prof in (ncp.sweep_profile, ncp.sweep_profile_direct):
        order, cut, vol, phi = prof(g, [0.4, 0.3, 0.2, 0.1])
        assert order.tolist() == [0, 1, 2, 3]
        assert cut.tolist() == [4, 4, 4, 0] and vol.tolist() == [4, 8, 12, 16]
        assert phi[:3].tolist() == [1.0, 0.5, 1.0] and np.isinf(phi[3])
    assert ncp.best_cut(phi) == (2, 0.5)


@pytest.mark.parametrize("m", [3, 5, 8])
def test_two_cliques_and_a_bridge(m):
    s, t = [], []
    for base in (0, m):
        for i in range(m):
            for j in range(m):
                if i != j:
                    s.append(base + i)
                    t.append(base + j)
    s += [0, m]
    t += [m, 0]  # the bridge, both directions
    g = fi.from_edges(2 * m, s, t)
    p = np.zeros(2 * m, np.float32)
    p[:m] = np.linspace(1.0, 0.5, m)  # mass on the first clique, a little on the second
    p[m:] = np.linspace(0.01, 0.001, m)
    order, cut, vol, phi = ncp.sweep_profile(g, p)
    k, best = ncp.best_cut(phi)
    assert k == m and sorted(order[:m].tolist()) == list(range(m))
    assert cut[m - 1] == 2 and vol[m - 1] == 2 * m * (m - 1) + 2
    assert best == pytest.approx(1.0 / (m * (m - 1) + 1))


@pytest.mark.parametrize("seed", range(6))
def test_incremental_equals_the_definition(seed):
    rng = np.random.default_rng(seed)
    g = fi.random_small(int(rng.integers(5, 60)), int(rng.integers(5, 300)), seed, weighted=False)
    p = rng.random(g.num_vertices).astype(np.float32)
    p[rng.random(g.num_vertices) < 0.3] = 0.0  # outside the support
    if seed % 2:
        p[: g.num_vertices // 2] = 0.25  # many equal keys among equal degrees
    pos = rng.permutation(g.num_vertices) if seed % 3 == 0 else None
    for max_size in (None, 1, 7):
        a = ncp.sweep_profile(g, p, max_size, pos)
        b = ncp.sweep_profile_direct(g, p, max_size, pos)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_sweep_order_ties_support_and_truncation():
    g = fi.from_edges(5, [0, 1, 2, 3, 4, 0], [1, 2, 3, 4, 0, 0])  # a 5-cycle plus a self-loop at 0
    d = ncp.degrees(g)
    assert d.tolist() == [4, 2, 2, 2, 2]
    p = np.array([0.8, 0.1, 0.1, 0.1, 0.0], np.float32)  # 0: key 0.2; 1-3: key 0.05 each; 4 outside
    assert ncp.sweep_order(g, p).tolist() == [0, 1, 2, 3]
    assert ncp.sweep_order(g, p, pos=[0, 3, 2, 1, 4]).tolist() == [0, 3, 2, 1]  # ties by position
    assert ncp.sweep_order(g, p, max_size=2).tolist() == [0, 1]
    iso = fi.from_edges(3, [0], [1])  # vertex 2 has no edges: never in a sweep
    assert ncp.sweep_order(iso, [0.5, 0.2, 0.3]).tolist() == [0, 1]


def test_ncp_takes_the_least_conductance_per_size_range():
    phis = [np.array([0.9, 0.5, 0.7, 0.4]), np.array([0.8, 0.6]), np.array([np.inf, 0.2, 0.3, 0.35, 0.1])]
    best = ncp.ncp(phis, 5)
    # sizes 1 | 2-3 | 4-7
    assert best.tolist() == [0.8, 0.2, 0.1]
