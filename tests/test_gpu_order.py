"""GPU parity with a caller-supplied vertex order: the library relabels the
graph internally, and sources, result vectors (host and device) and digests
stay in the caller's ids, bit-exact against the oracle."""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle
from digests import sp_digest
from paper_2103_14915_amd import order

pytestmark = pytest.mark.gpu

ALPHA = 0.15


def _fork():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_14915_amd as fork
    return fork


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("seed,pv", [(1, 8), (2, 64), (3, 1024)])
def test_random_order_sssp_bfs_ppr_in_caller_ids(seed, pv):
    import torch
    fork = _fork()
    g = fi.random_small(300, 2400, seed, wmax=50)
    pos = np.random.default_rng(100 + seed).permutation(g.num_vertices).astype(np.uint32)
    s_sp = fi.sources_uniform(g, 10, 200 + seed)
    s_pr = fi.sources_uniform(g, 6, 300 + seed)
    say("order seed", seed, "pv", pv)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=pv, vertex_order=pos)
    a = fg.submit("sssp", s_sp)
    b = fg.submit("bfs", s_sp)
    c = fg.submit("ppr", s_pr, alpha=ALPHA, epsilon=1e-6, eps_mode=0)
    fg.run(max_passes=200000)
    ref_sp, ref_bf = oracle.sssp(g, s_sp), oracle.bfs(g, s_sp)
    for i in range(len(s_sp)):
        np.testing.assert_array_equal(fg.fetch(a + i), ref_sp[i])
        np.testing.assert_array_equal(fg.fetch(b + i), ref_bf[i])
        d = fg.digest(a + i)
        assert (d["count"], d["sum"], d["hash"]) == sp_digest(ref_sp[i])
    # device destination
    out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
    fg.fetch(a, out=out)
    np.testing.assert_array_equal(out.cpu().numpy(), ref_sp[0])
    for i, s in enumerate(s_pr):
        p = fg.fetch(c + i, fork.FIELD_P).astype(np.float64)
        r = fg.fetch(c + i, fork.FIELD_R)
        assert oracle.push_terminal(g, r, 1e-6, 0, dtype=np.float32)
        assert oracle.ppr_invariant_l1(g, s, p, r.astype(np.float64), ALPHA) <= 1e-4
    parts = fg.partitions()
    assert parts[0] == 0 and parts[-1] == g.num_vertices  # internal positions
    fg.close()


def test_grid_tiles_match_row_major_results():
    fork = _fork()
    g = fi.grid(128, 96, weights=(1, 1000), weight_seed=9)
    pos = order.grid_tiles(128, 96, 32)
    srcs = fi.sources_uniform(g, 16, 10)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=1024, vertex_order=pos)
    fg.submit("sssp", srcs)
    fg.submit("bfs", srcs)
    fg.run(max_passes=200000)
    ref_sp, ref_bf = oracle.sssp(g, srcs), oracle.bfs(g, srcs)
    for i in range(len(srcs)):
        np.testing.assert_array_equal(fg.fetch(i), ref_sp[i])
        np.testing.assert_array_equal(fg.fetch(len(srcs) + i), ref_bf[i])
    assert len(fg.partitions()) - 1 == 128 * 96 // 1024  # one 32 x 32 tile per partition
    fg.close()


def test_vertex_order_on_device_and_rejected_orders():
    import torch
    fork = _fork()
    g = fi.random_small(200, 1000, 7, wmax=20)
    pos = np.random.default_rng(8).permutation(g.num_vertices).astype(np.uint32)
    srcs = fi.sources_uniform(g, 5, 9)
    t = lambda x, dt: torch.as_tensor(np.asarray(x).astype(dt), device="cuda")
    fg = fork.ForkGraph(g.num_vertices, t(g.row_ptr, np.int64), t(g.col, np.int32), t(g.weight, np.int32),
                        partition_vertices=32, vertex_order=t(pos, np.int32))
    fg.submit("sssp", srcs)
    fg.run(max_passes=200000)
    ref = oracle.sssp(g, srcs)
    for i in range(len(srcs)):
        np.testing.assert_array_equal(fg.fetch(i), ref[i])
    fg.close()
    bad_dup = pos.copy()
    bad_dup[1] = bad_dup[0]
    bad_range = pos.copy()
    bad_range[3] = g.num_vertices
    for bad in (bad_dup, bad_range, pos[:-1].copy()[np.r_[0:len(pos) - 1, 0]]):
        with pytest.raises(fork.ForkError) as e:
            fork.ForkGraph.from_graph(g, vertex_order=bad)
        assert e.value.code == fork.FORK_E_INVALID
