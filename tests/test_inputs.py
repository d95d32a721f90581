"""Checks of the seeded input generators (shape, determinism, distribution)."""
import numpy as np

import fpp_inputs as fi


def test_rmat_shape_and_determinism():
    g1 = fi.rmat(10, seed=3, weights=(1, 255), weight_seed=5)
    g2 = fi.rmat(10, seed=3, weights=(1, 255), weight_seed=5)
    assert g1.num_vertices == 1024 and g1.num_edges == 16 * 1024
    np.testing.assert_array_equal(g1.col, g2.col)
    np.testing.assert_array_equal(g1.weight, g2.weight)
    assert g1.weight.min() >= 1 and g1.weight.max() <= 255
    assert np.all(np.diff(g1.row_ptr.astype(np.int64)) >= 0)


def test_rmat_quadrant_frequencies():
    # the top bit of (src, dst) follows (a, b, c, d)
    g = fi.rmat(14, seed=11)
    src = np.repeat(np.arange(g.num_vertices), g.out_degree())
    hs, hd = src >> 13, g.col.astype(np.int64) >> 13
    n = g.num_edges
    freq = [np.count_nonzero((hs == i) & (hd == j)) / n for i, j in ((0, 0), (0, 1), (1, 0), (1, 1))]
    np.testing.assert_allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.01)


def test_grid_counts_and_symmetric_weights():
    g = fi.grid(2048, 2048)
    assert g.num_vertices == 4194304 and g.num_edges == 16769024
    g = fi.grid(5, 6, weights=(1, 1000), weight_seed=2)
    src = np.repeat(np.arange(30), g.out_degree())
    w = {(int(s), int(d)): int(x) for s, d, x in zip(src, g.col, g.weight)}
    for (s, d), x in w.items():
        assert w[(d, s)] == x
        r1, c1 = divmod(s, 6)
        r2, c2 = divmod(d, 6)
        assert abs(r1 - r2) + abs(c1 - c2) == 1


def test_sources():
    g = fi.rmat(12, seed=1)
    s = fi.sources_uniform(g, 64, 9)
    assert len(set(s.tolist())) == 64 and np.all(g.out_degree()[s] > 0)
    top = set(fi.top_degree_set(g).tolist())
    assert len(top) == 41
    m = fi.sources_mixed(g, 40, 3)
    assert all(int(v) in top for v in m[1::2])
