"""GPU betweenness centrality (fork_bc) against the oracle's Brandes sweeps
(oracle/bc.py, pinned by brute-force path enumeration and closed forms),
on the same BFS or SSSP sources.  The oracle's path counts are exact integers
in fp64; the GPU keeps their logarithms, so each ratio carries a relative
rounding error of a few 1e-16 per DAG edge: rtol 1e-9."""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
from oracle import bc

pytestmark = pytest.mark.gpu


def _fork():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_14915_amd as fork
    return fork


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind,ordered,qt", [("rmat", False, "bfs"), ("rmat", True, "bfs"), ("grid", False, "bfs"),
                                            ("rmat_w", False, "sssp"), ("rmat_w", True, "sssp"),
                                            ("grid_w", False, "sssp")])
def test_bc_matches_brandes(kind, ordered, qt):
    """BFS sources (unit steps) and SSSP sources on weighted graphs (the
    shortest-path DAG of the weights), with and without a vertex order."""
    fork = _fork()
    g = {"rmat": lambda: fi.rmat(10, seed=91), "grid": lambda: fi.grid(96, 96, weights=None),
         "rmat_w": lambda: fi.rmat(10, seed=91, weights=(1, 4), weight_seed=96),
         "grid_w": lambda: fi.grid(48, 48, weights=(1, 3), weight_seed=97)}[kind]()
    srcs = fi.sources_uniform(g, 10, 92)
    pos = np.random.default_rng(93).permutation(g.num_vertices).astype(np.uint32) if ordered else None
    say("bc", kind, "ordered", ordered, qt)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=512, vertex_order=pos)
    fg.submit("bfs" if qt == "sssp" else "sssp", srcs[:2])  # other queries in the batch are ignored by fork_bc
    first = fg.submit(qt, srcs)
    fg.run(max_passes=400000)
    got = fg.bc(first, len(srcs))
    fg.close()
    ref = bc.centrality(g, srcs, unit=qt == "bfs")
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9)
    assert ref.max() > 0


def test_bc_errors():
    fork = _fork()
    g = fi.rmat(9, seed=94)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=128, max_queries=4)
    a = fg.submit("ppr", [1, 2])
    b = fg.submit("bfs", fi.sources_uniform(g, 8, 95))
    with pytest.raises(fork.ForkError) as e:
        fg.bc(b, 1)
    assert e.value.code == fork.FORK_E_STATE  # not run yet
    fg.run(max_passes=200000)
    for args, code in (((a, 1), fork.FORK_E_INVALID), ((b, 100), fork.FORK_E_INVALID),  # PPR; out of range
                       ((b, 1), fork.FORK_E_STATE)):  # the first BFS queries ran in an earlier wave
        with pytest.raises(fork.ForkError) as e:
            fg.bc(*args)
        assert e.value.code == code, args
    last = len(fg.types) - 1
    one = fg.bc(last, 1)
    assert one.shape == (g.num_vertices,) and np.all(one >= 0)
    assert np.all(fg.bc(last, 0) == 0)
    fg.close()


@pytest.mark.parametrize("n", [640, 2048])
def test_bc_on_a_grid_whose_path_counts_overflow_fp64(n):
    """On an n x n grid a corner has C(2n - 2, n - 1) shortest paths to the
    opposite corner: about 10^383 for n = 640 and 10^1231 for n = 2048, far
    beyond fp64.  Logarithmic counts stay finite, and the total is fixed:
    every shortest s-t path of unit-weight edges has d(s, t) - 1 interior
    vertices, so the dependencies summed over all vertices give the sum over
    t of (d(s, t) - 1) per source.  A corner source also makes the result
    symmetric under transposing the grid.  The levels come from the
    oracle's BFS."""
    import oracle
    fork = _fork()
    g = fi.grid(n, n, weights=None)
    srcs = np.array([0, n - 1, n * n - 1, (n // 2) * n + n // 3], np.uint32)  # three corners and an inner vertex
    fg = fork.ForkGraph.from_graph(g, partition_vertices=8192)
    first = fg.submit("bfs", srcs)
    fg.run(max_passes=400000)
    got = fg.bc(first, len(srcs))
    corner = fg.bc(first, 1)  # from (0, 0) alone
    fg.close()
    assert np.all(np.isfinite(got)) and np.all(got >= 0)
    lv = oracle.bfs(g, srcs).astype(np.int64)
    expect = float(sum(np.sum(lv[i][lv[i] > 0] - 1) for i in range(len(srcs))))
    assert got.sum() == pytest.approx(expect, rel=1e-9)
    c2 = corner.reshape(n, n)
    np.testing.assert_allclose(c2, c2.T, rtol=1e-9, atol=1e-6)
    assert corner.sum() == pytest.approx(float(np.sum(lv[0][lv[0] > 0] - 1)), rel=1e-9)


def test_bc_value_range_error():
    """SSSP distances on a 300 x 300 grid with weights up to 1,000 span more
    than the 65,536 values fork_bc sorts by: FORK_E_CAPACITY, and nothing is
    written."""
    fork = _fork()
    g = fi.grid(300, 300, weights=(1, 1000), weight_seed=98)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=8192)
    first = fg.submit("sssp", [0])
    fg.run(max_passes=400000)
    assert fg.fetch(first).max() > 65536
    with pytest.raises(fork.ForkError) as e:
        fg.bc(first, 1)
    assert e.value.code == fork.FORK_E_CAPACITY
    fg.close()
