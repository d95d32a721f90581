"""GPU parity of the grouped engine (64 queries of one type per work item,
vertex-major state rows) against the CPU oracle: SSSP/BFS bit-exact, PPR
within the push gates (termination in fp32, invariant <= 1e-4 L1, p, r >= 0),
over partial groups, partition sizes, schedulers, waves and vertex orders."""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle

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


def check_ppr(fork, fg, g, srcs, first, eps, mode):
    for i, s in enumerate(srcs):
        p = fg.fetch(first + i, fork.FIELD_P)
        r = fg.fetch(first + i, fork.FIELD_R)
        assert np.all(p >= 0) and np.all(r >= 0)
        assert oracle.push_terminal(g, r, eps, mode, dtype=np.float32), i
        assert oracle.ppr_invariant_l1(g, s, p.astype(np.float64), r.astype(np.float64), ALPHA) <= 1e-4, i


@pytest.mark.parametrize("weights,seed", [((1, 1_000_000), 91), (None, 93)])
def test_grouped_sssp_other_weight_widths(weights, seed):
    """R-MAT 13 SSSP on the grouped engine with 4-byte weights (up to 10^6)
    and on an unweighted graph (unit weights): bit-exact, with a partial
    group, at 1,024 threads per workgroup as the tuned runs use."""
    fork = _fork()
    g = fi.rmat(13, seed=seed, weights=weights, weight_seed=seed + 1) if weights else fi.rmat(13, seed=seed)
    srcs = fi.sources_uniform(g, 100, seed + 2)
    say("grouped sssp weights", weights)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=1024)
    fg.submit("sssp", srcs)
    fg.run(engine="grouped", group_threads=1024, max_passes=200000)
    st = fg.stats()
    d = np.stack([fg.fetch(i) for i in range(len(srcs))])
    fg.close()
    assert st["weight_bytes"] == (4 if weights else 0), st["weight_bytes"]
    np.testing.assert_array_equal(d, oracle.sssp(g, srcs))


@pytest.mark.parametrize("pv,sched", [(64, "priority"), (512, "priority"), (4096, "fifo"), (16384, "random"),
                                      (512, "maxops")])
def test_grouped_mixed_batch_exact(pv, sched):
    """R-MAT 13 (8,192 vertices): from 128 partitions down to a single one."""
    fork = _fork()
    g = fi.rmat(13, seed=71, weights=(1, 255), weight_seed=72)
    s_sp = fi.sources_uniform(g, 100, 1)   # one full group and one partial
    s_bfs = fi.sources_uniform(g, 70, 2)
    s_pr = fi.sources_uniform(g, 50, 3)
    say("grouped mixed pv", pv, sched)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=pv)
    fg.submit("sssp", s_sp)
    fg.submit("bfs", s_bfs)
    fg.submit("ppr", s_pr, alpha=ALPHA, epsilon=1e-6, eps_mode=1)
    fg.run(engine="grouped", scheduler=sched, max_passes=200000)
    d = np.stack([fg.fetch(i) for i in range(100)])
    lv = np.stack([fg.fetch(100 + i) for i in range(70)])
    np.testing.assert_array_equal(d, oracle.sssp(g, s_sp))
    np.testing.assert_array_equal(lv, oracle.bfs(g, s_bfs))
    check_ppr(fork, fg, g, s_pr, 170, 1e-6, 1)
    st = fg.stats()
    assert st["edges"] > 0 and st["work_items"] > 0
    fg.close()


@pytest.mark.parametrize("mode,eps", [(0, 1e-5), (1, 1e-6)])
def test_grouped_ppr_threshold_modes(mode, eps):
    fork = _fork()
    g = fi.rmat(13, seed=73)
    srcs = fi.sources_uniform(g, 64, 4)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=1024)
    fg.submit("ppr", srcs, alpha=ALPHA, epsilon=eps, eps_mode=mode)
    fg.run(engine="grouped")
    check_ppr(fork, fg, g, srcs, 0, eps, mode)
    fg.close()


def test_grouped_grid_sssp_and_bfs_exact():
    """High diameter: a 96 x 96 weighted grid (many passes, windows matter)."""
    fork = _fork()
    g = fi.grid(96, 96, weights=(1, 1000), weight_seed=5)
    s_sp = fi.sources_uniform(g, 64, 6)
    s_bfs = fi.sources_uniform(g, 16, 7)
    for window, delta in ((0, 0), (16, 4000)):
        fg = fork.ForkGraph.from_graph(g, partition_vertices=1024)
        fg.submit("sssp", s_sp)
        fg.submit("bfs", s_bfs)
        fg.run(engine="grouped", window=window, delta=delta)
        np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(64)]), oracle.sssp(g, s_sp))
        np.testing.assert_array_equal(np.stack([fg.fetch(64 + i) for i in range(16)]), oracle.bfs(g, s_bfs))
        fg.close()


def test_grouped_waves_digests_and_vertex_order():
    """More queries than one wave holds: every query gets a digest equal to the
    buffered engine's, the last wave keeps vectors; a vertex order relabels."""
    fork = _fork()
    g = fi.rmat(11, seed=75, weights=(1, 255), weight_seed=76)
    srcs = fi.sources_uniform(g, 200, 8)
    order = np.random.default_rng(9).permutation(g.num_vertices).astype(np.uint32)
    digs = []
    for engine in ("buffered", "grouped"):
        fg = fork.ForkGraph.from_graph(g, partition_vertices=256, max_queries=80, vertex_order=order)
        fg.submit("sssp", srcs)
        fg.run(engine=engine)
        digs.append([(fg.digest(i)["hash"], fg.digest(i)["count"], fg.digest(i)["sum"]) for i in range(200)])
        if engine == "grouped":
            assert fg.stats()["waves"] == 3
            np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(160, 200)]),
                                          oracle.sssp(g, srcs[160:200]))
        fg.close()
    assert digs[0] == digs[1]


def test_prepare_allocates_without_running():
    """fork_prepare sizes the buffers for the largest of waves that mix query
    types differently (SSSP only, both, PPR only), runs nothing (fetch still
    reports FORK_E_STATE), and the run after it is exact."""
    fork = _fork()
    g = fi.rmat(11, seed=79, weights=(1, 255), weight_seed=80)
    s_sp = fi.sources_uniform(g, 100, 10)
    s_pr = fi.sources_uniform(g, 100, 11)
    digs = []
    for prep in (True, False):
        fg = fork.ForkGraph.from_graph(g, partition_vertices=512, max_queries=80)
        fg.submit("sssp", s_sp)
        fg.submit("ppr", s_pr, alpha=ALPHA, epsilon=1e-5, eps_mode=1)
        if prep:
            fg.prepare(engine="grouped", group_threads=1024)
            with pytest.raises(fork.ForkError) as e:
                fg.fetch(0)
            assert e.value.code == fork.FORK_E_STATE
        fg.run(engine="grouped", group_threads=1024)
        assert fg.stats()["waves"] == 3
        digs.append([(fg.digest(i)["hash"], fg.digest(i)["count"]) for i in range(100)])
        fg.close()
    assert digs[0] == digs[1]
    ref = oracle.sssp(g, s_sp)
    assert all(digs[0][i][1] == int(np.sum(ref[i] != np.int32(0x7FFFFFFF))) for i in range(100))


def test_grouped_learned_scheduler_exact():
    fork = _fork()
    g = fi.rmat(12, seed=77, weights=(1, 255), weight_seed=78)
    srcs = fi.sources_uniform(g, 64, 9)
    theta = np.load(fork.__file__.replace("__init__.py", "sched_mlp.npy"))
    fg = fork.ForkGraph.from_graph(g, partition_vertices=256)
    fg.submit("sssp", srcs)
    fg.run(engine="grouped", scheduler="learned", mlp_weights=theta)
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(64)]), oracle.sssp(g, srcs))
    fg.close()


def test_grouped_rejects_what_it_does_not_run():
    fork = _fork()
    g = fi.rmat(9, seed=79)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=256)
    fg.submit("ppr", fi.sources_uniform(g, 4, 1), alpha=ALPHA, epsilon=1e-6, l1_target=1e-4)
    with pytest.raises(fork.ForkError) as e:
        fg.run(engine="grouped")
    assert e.value.code == fork.FORK_E_INVALID
    fg.close()
    fg = fork.ForkGraph.from_graph(g, partition_vertices=256)
    fg.submit("bfs", fi.sources_uniform(g, 4, 1))
    for kw in (dict(persistent=1), dict(trace=1), dict(engine=7)):
        with pytest.raises(fork.ForkError) as e:
            fg.run(**dict(dict(engine="grouped"), **kw))
        assert e.value.code == fork.FORK_E_INVALID
    fg.run(engine="grouped")  # still usable
    np.testing.assert_array_equal(fg.fetch(0), oracle.bfs(g, fi.sources_uniform(g, 4, 1))[0])
    fg.close()
