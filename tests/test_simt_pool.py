"""The library's kernels run on the CPU (tests/simt: a host stand-in for the
HIP runtime in which workgroups are OS threads and lanes are coroutines),
with an ownership checker of the operation pool after every pass launch:
each chunk in exactly one place (free ring, one buffer's lists, one work
item), no cycles, counts matching, every buffered operation inside its
buffer's partition.

These runs drive the regimes that the GPU tests keep small: a free ring that
wraps many times, visits whose frontier overflows so that activated vertices
are retained as operations in the visit's own buffer, hashed slices whose
probe paths fill up, certified-PPR refinements on partitions larger than the
frontier, and the persistent kernel.  The checker itself is shown to see
planted mistakes (a double free, a lost chunk, a misrouted chunk, a wrong
count), each planted in a run of its own.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle
from digests import sp_digest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests", "simt"))

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def fs():
    import fork_simt
    fork_simt.load()
    return fork_simt


def _clean(fs, lib):
    c = fs.checker(lib)
    assert c["checks"] > 0
    assert c["failures"] == 0, c["message"]
    return c


def test_sssp_and_bfs_exact_with_a_wrapping_free_ring(fs):
    """A pool of 1,527 chunks reused many times over.  How many chunks are
    held at once depends on how the workgroups interleave, so a run may also
    split the queries into waves when the pool runs out (then only the last
    wave's vectors stay resident): every query's digest is checked, and the
    vectors of the resident ones."""
    import paper_2103_14915_amd as fork
    lib = fs.load()
    fs.reset_checker(lib)
    g = fi.rmat(11, seed=21, weights=(1, 255), weight_seed=22)
    s_sp = fi.sources_uniform(g, 16, 1)
    s_bfs = fi.sources_uniform(g, 8, 2)
    ref = list(oracle.sssp(g, s_sp)) + list(oracle.bfs(g, s_bfs))
    fg = fs.SimtGraph(lib, g, partition_vertices=128, pool_bytes=3 << 20)  # 1,527 chunks
    fg.submit("sssp", s_sp)
    fg.submit("bfs", s_bfs)
    fg.run(max_passes=100000)
    st = fg.stats()
    resident = 0
    for i in range(24):
        d = fg.digest(i)
        assert (d["count"], d["sum"], d["hash"]) == sp_digest(ref[i]), i
        try:
            got = fg.fetch(i)
        except fork.ForkError as e:  # not resident
            assert e.code == fork.FORK_E_STATE and st["waves"] > 1, i
            continue
        resident += 1
        np.testing.assert_array_equal(got, ref[i], err_msg=f"query {i}")
    fg.close()
    assert resident >= 1 and (resident == 24) == (st["waves"] == 1)
    assert st["chunks"] > 2 * 1527  # the pool's chunks were reused more than twice
    _clean(fs, lib)


def test_persistent_kernel_exact_and_consistent(fs):
    lib = fs.load()
    fs.reset_checker(lib)
    g = fi.rmat(10, seed=23, weights=(1, 255), weight_seed=24)
    srcs = fi.sources_uniform(g, 8, 3)
    fg = fs.SimtGraph(lib, g, partition_vertices=128, pool_bytes=4 << 20)
    fg.submit("sssp", srcs)
    fg.run(max_passes=100000, persistent=1)
    d = np.stack([fg.fetch(i) for i in range(8)])
    fg.close()
    np.testing.assert_array_equal(d, oracle.sssp(g, srcs))
    _clean(fs, lib)


def test_ppr_frontier_spill_and_hash_fallback(fs):
    """2,048-vertex partitions (twice the frontier) with 256 hash slots and a
    small threshold: visits retain activated vertices as operations in their
    own buffer, and most vertices live outside the LDS table."""
    lib = fs.load()
    fs.reset_checker(lib)
    g = fi.rmat(11, seed=31)
    srcs = fi.sources_uniform(g, 4, 32)
    eps = 1e-8
    fg = fs.SimtGraph(lib, g, partition_vertices=2048, pool_bytes=16 << 20)
    fg.submit("ppr", srcs, epsilon=eps, eps_mode=0)
    fg.run(max_passes=100000, slice_slots=256)
    st = fg.stats()
    P = [fg.fetch(i, 1).astype(np.float64) for i in range(4)]
    R = [fg.fetch(i, 2) for i in range(4)]
    fg.close()
    assert st["spilled"] > 1000, st["spilled"]
    for i, s in enumerate(srcs):
        assert oracle.push_terminal(g, R[i], eps, 0, dtype=np.float32)
        assert oracle.ppr_invariant_l1(g, s, P[i], R[i].astype(np.float64), 0.15) <= 1e-4
    _clean(fs, lib)


def test_certified_refinement_on_partitions_larger_than_the_frontier(fs):
    """The certified mode's refinement re-activates most of a 4,096-vertex
    partition at once (the regime in which the GPU run failed): results meet
    the L1 target and the pool stays consistent."""
    lib = fs.load()
    fs.reset_checker(lib)
    g = fi.rmat(12, seed=31)
    srcs = fi.sources_uniform(g, 4, 32)
    fg = fs.SimtGraph(lib, g, partition_vertices=4096, pool_bytes=64 << 20)
    fg.submit("ppr", srcs, epsilon=1e-6, eps_mode=1, l1_target=1e-4)
    fg.run(max_passes=100000, slice_slots=256)
    st = fg.stats()
    P = np.stack([fg.fetch(i, 1) for i in range(4)]).astype(np.float64)
    R = np.stack([fg.fetch(i, 2) for i in range(4)]).astype(np.float64)
    fg.close()
    assert st["refine_rounds"] >= 1 and st["spilled"] > 1000, st
    pi = oracle.ppr_exact(g, srcs, 0.15)
    for i in range(4):
        assert R[i].sum() <= 0.9e-4 * (1 + 1e-6)
        assert np.abs(P[i] - pi[i]).sum() <= 1e-4
    _clean(fs, lib)


@pytest.mark.parametrize("plant,expect", [("dup", "already owned"), ("leak", "owned by nothing"),
                                          ("misroute", "outside partition"), ("count", "bcnt")])
def test_checker_sees_planted_mistakes(fs, plant, expect):
    env = dict(os.environ, SIMT_PLANT=plant)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "simt", "fork_simt.py"), "sssp_small_pool"],
                       env=env, capture_output=True, text=True, timeout=300, cwd=ROOT)
    line = [x for x in r.stdout.splitlines() if x.startswith("{")]
    assert line, (r.returncode, r.stderr[-2000:])
    c = json.loads(line[-1])["check"]
    assert c["failures"] >= 1 and expect in c["message"], c


def test_grouped_engine_exact_under_concurrency(fs):
    """The grouped engine on the host (real concurrency between workgroups):
    SSSP/BFS bit-exact and PPR within the push gates, with a partial group."""
    lib = fs.load()
    g = fi.rmat(10, seed=21, weights=(1, 255), weight_seed=22)
    s_sp = fi.sources_uniform(g, 70, 1)
    s_bfs = fi.sources_uniform(g, 10, 2)
    s_pr = fi.sources_uniform(g, 20, 3)
    fg = fs.SimtGraph(lib, g, partition_vertices=128)
    fg.submit("sssp", s_sp)
    fg.submit("bfs", s_bfs)
    fg.submit("ppr", s_pr, epsilon=1e-6, eps_mode=0)
    fg.run(max_passes=100000, engine="grouped")
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(70)]), oracle.sssp(g, s_sp))
    np.testing.assert_array_equal(np.stack([fg.fetch(70 + i) for i in range(10)]), oracle.bfs(g, s_bfs))
    for i, s in enumerate(s_pr):
        p = fg.fetch(80 + i, 1).astype(np.float64)
        r = fg.fetch(80 + i, 2)
        assert np.all(p >= 0) and np.all(r >= 0)
        assert oracle.push_terminal(g, r, 1e-6, 0, dtype=np.float32)
        assert oracle.ppr_invariant_l1(g, s, p, r.astype(np.float64), 0.15) <= 1e-4
    fg.close()


@pytest.mark.parametrize("weights,seed", [((1, 1_000_000), 91), (None, 93)])
def test_grouped_engine_other_weight_widths(fs, weights, seed):
    """The grouped engine's SSSP edge steps with 4-byte weights (up to 10^6,
    where the relaxed sum needs the overflow test) and on an unweighted graph
    (unit weights), on the host with real concurrency: bit-exact, with a
    partial group."""
    lib = fs.load()
    g = fi.rmat(10, seed=seed, weights=weights, weight_seed=seed + 1) if weights else fi.rmat(10, seed=seed)
    srcs = fi.sources_uniform(g, 70, seed + 2)
    fg = fs.SimtGraph(lib, g, partition_vertices=128)
    fg.submit("sssp", srcs)
    fg.run(max_passes=100000, engine="grouped")
    st = fg.stats()
    d = np.stack([fg.fetch(i) for i in range(len(srcs))])
    fg.close()
    assert st["weight_bytes"] == (4 if weights else 0), st["weight_bytes"]
    np.testing.assert_array_equal(d, oracle.sssp(g, srcs))


def test_no_alloc_training_on_the_host_build(fs):
    """fork_mlp_train_noalloc against fork_mlp_train in the host build (where
    device pointers are host pointers): two calls in a row, the second with
    fewer samples, reuse the library's fixed scratch array."""
    import ctypes
    from oracle import mlp as omlp
    lib = fs.load()
    P, U32, U64, F = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float
    lib.fork_mlp_train.argtypes = [P, P, P, U64, U32, U32, F, U64, P]
    lib.fork_mlp_train_noalloc.argtypes = [P, P, P, U64, U32, U32, F, U64, P, P]
    rng = np.random.default_rng(21)
    theta0 = omlp.init(13).astype(np.float32)
    for n, steps, batch, lr, seed in ((3000, 7, 256, 3e-3, 5), (500, 4, 128, 1e-3, 6)):
        x = rng.normal(size=(n, 16)).astype(np.float32)
        t = (x[:, 0] - np.abs(x[:, 1])).astype(np.float32)
        a, b = theta0.copy(), theta0.copy()
        la, lb = np.zeros(steps, np.float32), np.full(steps, 123.0, np.float32)
        assert lib.fork_mlp_train(a.ctypes.data, x.ctypes.data, t.ctypes.data, n, steps, batch, lr, seed,
                                  la.ctypes.data) == 0
        assert lib.fork_mlp_train_noalloc(b.ctypes.data, x.ctypes.data, t.ctypes.data, n, steps, batch, lr, seed,
                                          lb.ctypes.data, None) == 0
        np.testing.assert_allclose(lb, la, rtol=1e-5, atol=1e-7)
        d = np.abs(a.astype(np.float64) - b)
        assert np.mean(d <= 1e-6 + 1e-5 * np.abs(a)) >= 0.995
    big = np.zeros((32769, 16), np.float32)
    assert lib.fork_mlp_train_noalloc(theta0.ctypes.data, big.ctypes.data, big[:, 0].copy().ctypes.data, 32769, 1,
                                      256, 1e-3, 0, None, None) == -1


def test_prepare_leaves_nothing_to_allocate_for_the_run(fs):
    """fork_prepare allocates every device buffer of a grouped run whose waves
    mix query types differently (PPR only, both, SSSP only); the runs after it
    allocate nothing, and the last wave's SSSP vectors are exact."""
    import ctypes
    import paper_2103_14915_amd as fork
    lib = fs.load()
    lib.simt_alloc_calls.restype = ctypes.c_uint64
    lib.fork_prepare.argtypes = [ctypes.c_void_p, ctypes.POINTER(fork.fork_run_opts)]
    lib.fork_prepare.restype = ctypes.c_int
    g = fi.rmat(10, seed=79, weights=(1, 255), weight_seed=80)
    s_sp, s_pr = fi.sources_uniform(g, 100, 10), fi.sources_uniform(g, 100, 11)
    ref = oracle.sssp(g, s_sp[60:])
    for prep in (True, False):
        sg = fs.SimtGraph(lib, g, partition_vertices=256, max_queries=80)
        sg.submit("ppr", s_pr, alpha=0.15, epsilon=1e-4, eps_mode=1)
        sg.submit("sssp", s_sp)
        o = fork.fork_run_opts()
        o.engine, o.group_threads = fork.ENGINES["grouped"], 256
        if prep:
            assert lib.fork_prepare(sg.ctx, ctypes.byref(o)) == 0
            n0 = lib.simt_alloc_calls()
            assert lib.fork_run(sg.ctx, ctypes.byref(o)) == 0
            assert lib.fork_run(sg.ctx, ctypes.byref(o)) == 0
            assert lib.simt_alloc_calls() == n0
        else:
            assert lib.fork_run(sg.ctx, ctypes.byref(o)) == 0
        assert sg.stats()["waves"] == 3
        # the last wave (the last 40 SSSP queries) keeps its vectors
        np.testing.assert_array_equal(np.stack([sg.fetch(160 + i) for i in range(40)]), ref)
        sg.close()
