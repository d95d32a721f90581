"""Vertex orders for locality-aware partitions.

The library cuts the graph into contiguous ranges of its internal vertex
numbering (Definition 2.1).  An order that keeps neighbours close together
makes partitions with fewer cut edges, so fewer operations cross partitions
and queries settle in fewer passes.  The paper partitions with METIS and
reports a large gain over random partitions (Appendix C, effects of partition and cache size).  These helpers
give the position of each vertex in such an order, for
``ForkGraph(..., vertex_order=pos)``.  They only change speed: results are
the same for any order.

- ``grid_tiles``: 2D tiles of a row-major grid, row-major inside each tile.
  A tile of as many vertices as a partition makes each partition a square
  block, with 4·side cut edges instead of the 2·cols of a band of rows.
- ``rcm``: reverse Cuthill-McKee (scipy) on the symmetrised graph, a
  bandwidth-reducing order for general sparse graphs.
"""
from __future__ import annotations

import math

import numpy as np


def identity(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.uint32)


def grid_tiles(rows: int, cols: int, tile_rows: int, tile_cols: int = 0) -> np.ndarray:
    """Position of vertex r*cols + c when the grid is numbered tile by tile
    (tiles row-major, vertices row-major inside a tile; edge tiles may be
    smaller)."""
    tile_cols = tile_cols or tile_rows
    if rows <= 0 or cols <= 0 or tile_rows <= 0 or tile_cols <= 0:
        raise ValueError("grid and tile sizes must be positive")
    r = np.repeat(np.arange(rows, dtype=np.int64), cols)
    c = np.tile(np.arange(cols, dtype=np.int64), rows)
    order = np.lexsort((c, r, c // tile_cols, r // tile_rows))  # vertices in tile order
    pos = np.empty(rows * cols, np.uint32)
    pos[order] = np.arange(rows * cols, dtype=np.uint32)
    return pos


def square_tile(partition_vertices: int) -> int:
    """Side of the square tile with at most partition_vertices vertices."""
    return max(1, int(math.isqrt(int(partition_vertices))))


def tile_shape(partition_vertices: int) -> tuple:
    """(rows, cols) of a tile that fills one partition: a power-of-two
    rectangle (square, or twice as wide as tall) when partition_vertices is a
    power of two, so tiles and partitions stay aligned; else the largest
    square."""
    pv = int(partition_vertices)
    if pv > 0 and pv & (pv - 1) == 0:
        k = pv.bit_length() - 1
        return 1 << (k // 2), 1 << (k - k // 2)
    s = square_tile(pv)
    return s, s


def rcm(g) -> np.ndarray:
    """Position of each vertex in the reverse Cuthill-McKee order of the
    symmetrised graph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    n = g.num_vertices
    rp = np.asarray(g.row_ptr, np.int64)
    a = sp.csr_matrix((np.ones(rp[-1], np.int8), np.asarray(g.col, np.int64), rp), shape=(n, n))
    perm = reverse_cuthill_mckee((a + a.T).tocsr(), symmetric_mode=True)
    pos = np.empty(n, np.uint32)
    pos[perm] = np.arange(n, dtype=np.uint32)
    return pos


def auto(spec: dict, g, partition_vertices: int):
    """The order the benchmark workloads use: tiles of one partition each
    for grids (their row-major numbering cuts a band of rows into each
    partition); None (the generator's numbering) for R-MAT graphs, whose
    vertices have no geometry."""
    if spec.get("kind") == "grid":
        return grid_tiles(spec["rows"], spec["cols"], *tile_shape(partition_vertices))
    return None
