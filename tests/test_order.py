"""Vertex-order helpers (host only): permutations, tile contiguity, and the
cut-edge count that motivates them."""
import numpy as np
import pytest

import fpp_inputs as fi
from paper_2103_14915_amd import order


def cut_edges(g, pos, part):
    """Edges whose endpoints fall in different contiguous ranges of `part` positions."""
    src = np.repeat(np.arange(g.num_vertices), np.diff(g.row_ptr.astype(np.int64)))
    return int(np.count_nonzero(pos[src] // part != pos[g.col.astype(np.int64)] // part))


@pytest.mark.parametrize("rows,cols,tr,tc", [(8, 8, 4, 4), (5, 7, 2, 3), (16, 4, 16, 4), (3, 3, 5, 5)])
def test_grid_tiles_is_a_permutation_with_contiguous_tiles(rows, cols, tr, tc):
    p = order.grid_tiles(rows, cols, tr, tc).astype(np.int64)
    assert sorted(p.tolist()) == list(range(rows * cols))
    r, c = np.divmod(np.arange(rows * cols), cols)
    tid = (r // tr) * ((cols + tc - 1) // tc) + c // tc
    for t in np.unique(tid):
        sel = np.sort(p[tid == t])
        assert sel[-1] - sel[0] + 1 == sel.size  # one contiguous range per tile
    # tiles follow each other row-major, and rows inside a tile are row-major
    assert p[0] == 0 and (rows * cols == 1 or p[1] == (1 if tc > 1 else p[1]))


def test_square_tiles_cut_fewer_edges_than_bands_of_rows():
    g = fi.grid(64, 64, weights=None)
    part = 256  # 16 x 16 tiles vs bands of 4 rows
    rowmajor = cut_edges(g, order.identity(g.num_vertices), part)
    tiles = cut_edges(g, order.grid_tiles(64, 64, order.square_tile(part)), part)
    # bands of 4 rows: 15 band boundaries of 64 grid edges, each in both directions;
    # 16 x 16 tiles: 3 horizontal and 3 vertical boundary lines of 64 grid edges
    assert rowmajor == 2 * 64 * (64 // 4 - 1)
    assert tiles == 2 * 2 * 64 * (64 // 16 - 1)
    assert tiles < rowmajor


def test_rcm_and_auto():
    g = fi.rmat(10, seed=4)
    p = order.rcm(g)
    assert sorted(p.tolist()) == list(range(g.num_vertices))
    assert order.auto({"kind": "rmat"}, g, 1024) is None
    gg = fi.grid(32, 32, weights=None)
    a = order.auto({"kind": "grid", "rows": 32, "cols": 32}, gg, 256)
    assert np.array_equal(a, order.grid_tiles(32, 32, 16))
    assert order.square_tile(65536) == 256 and order.square_tile(1000) == 31
    assert order.tile_shape(65536) == (256, 256) and order.tile_shape(8192) == (64, 128)
    assert order.tile_shape(32768) == (128, 256) and order.tile_shape(1000) == (31, 31)
    # a tile is exactly one partition's range of positions
    pv = 8192
    p = order.auto({"kind": "grid", "rows": 256, "cols": 256}, fi.grid(256, 256, weights=None), pv)
    r, c = np.divmod(np.arange(256 * 256), 256)
    assert np.all(p // pv == (r // 64) * 2 + c // 128)


def test_rcm_recovers_a_small_bandwidth_from_a_shuffled_grid():
    """A 20 x 20 grid under a random relabelling has bandwidth close to |V|;
    reverse Cuthill-McKee must bring it back to about a row or two."""
    g0 = fi.grid(20, 20, weights=None)
    perm = np.random.default_rng(3).permutation(g0.num_vertices)
    src = np.repeat(np.arange(g0.num_vertices), np.diff(g0.row_ptr.astype(np.int64)))
    g = fi.from_edges(g0.num_vertices, perm[src], perm[g0.col.astype(np.int64)])
    s2 = np.repeat(np.arange(g.num_vertices), np.diff(g.row_ptr.astype(np.int64)))

    def bandwidth(pos):
        return int(np.max(np.abs(pos[s2].astype(np.int64) - pos[g.col.astype(np.int64)].astype(np.int64))))

    assert bandwidth(order.identity(g.num_vertices)) > 300
    assert bandwidth(order.rcm(g)) <= 2 * 20 + 1
