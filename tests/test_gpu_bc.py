"""GPU betweenness centrality (fork_bc) against the oracle's Brandes sweeps
(oracle/bc.py, pinned by brute-force path enumeration and closed forms),
on the same BFS sources.  Path counts are integers, exact in fp64, and each
source's dependencies are summed in the same adjacency order on both sides;
only the order of the sum over sources differs, hence rtol 1e-12."""
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


@pytest.mark.parametrize("kind,ordered", [("rmat", False), ("rmat", True), ("grid", False)])
def test_bc_matches_brandes(kind, ordered):
    fork = _fork()
    if kind == "rmat":
        g = fi.rmat(10, seed=91)
    else:
        g = fi.grid(96, 96, weights=None)
    srcs = fi.sources_uniform(g, 10, 92)
    pos = np.random.default_rng(93).permutation(g.num_vertices).astype(np.uint32) if ordered else None
    say("bc", kind, "ordered", ordered)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=512, vertex_order=pos)
    fg.submit("sssp", srcs[:2])  # other queries in the batch are ignored by fork_bc
    first = fg.submit("bfs", srcs)
    fg.run(max_passes=400000)
    got = fg.bc(first, len(srcs))
    fg.close()
    ref = bc.centrality(g, srcs, unit=True)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)
    assert ref.max() > 0


def test_bc_errors():
    fork = _fork()
    g = fi.rmat(9, seed=94)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=128, max_queries=4)
    a = fg.submit("sssp", [1, 2])
    b = fg.submit("bfs", fi.sources_uniform(g, 8, 95))
    with pytest.raises(fork.ForkError) as e:
        fg.bc(b, 1)
    assert e.value.code == fork.FORK_E_STATE  # not run yet
    fg.run(max_passes=200000)
    for args, code in (((a, 1), fork.FORK_E_INVALID), ((b, 100), fork.FORK_E_INVALID),
                       ((b, 1), fork.FORK_E_STATE)):  # the first BFS queries ran in an earlier wave
        with pytest.raises(fork.ForkError) as e:
            fg.bc(*args)
        assert e.value.code == code, args
    last = len(fg.types) - 1
    one = fg.bc(last, 1)
    assert one.shape == (g.num_vertices,) and np.all(one >= 0)
    assert np.all(fg.bc(last, 0) == 0)
    fg.close()


def test_bc_on_a_grid_whose_path_counts_overflow_fp64():
    """On a 640 x 640 grid a corner has about 10^360 shortest paths to the
    opposite corner, beyond fp64, so plain path counts overflow.  The scaled
    counts must stay finite, and the total is fixed.  Every shortest s-t path
    of unit-weight edges has d(s, t) - 1 interior vertices, so summing the
    dependencies over all vertices gives sum over t of (d(s, t) - 1) per
    source.  The levels come from the oracle's BFS."""
    import oracle
    fork = _fork()
    n = 640
    g = fi.grid(n, n, weights=None)
    srcs = np.array([0, n - 1, n * n - 1, (n // 2) * n + n // 3], np.uint32)  # three corners and an inner vertex
    fg = fork.ForkGraph.from_graph(g, partition_vertices=8192)
    first = fg.submit("bfs", srcs)
    fg.run(max_passes=400000)
    got = fg.bc(first, len(srcs))
    fg.close()
    assert np.all(np.isfinite(got)) and np.all(got >= 0)
    lv = oracle.bfs(g, srcs).astype(np.int64)
    expect = float(sum(np.sum(lv[i][lv[i] > 0] - 1) for i in range(len(srcs))))
    assert got.sum() == pytest.approx(expect, rel=1e-9)
