"""GPU parity: the HIP fork-processing path against the CPU oracle.

SSSP and BFS must match bit-for-bit (int32, INT32_MAX = unreachable) and pass
the optimality certificate; PPR outputs must satisfy the push invariant
p + PPR(r) = PPR(e_s) within 1e-4 in L1 against fp64 power iteration, and the
termination rule max r/thr < 1, with p, r >= 0.
"""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle
from digests import sp_digest
from golden_io import load_sp_fixture

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


def run_sp(fork, g, srcs, qtype="sssp", sched="priority", **kw):
    load_kw = {k: kw.pop(k) for k in list(kw) if k in ("partition_vertices", "partition_edges", "pool_bytes",
                                                       "max_queries")}
    fg = fork.ForkGraph.from_graph(g, **load_kw)
    fg.submit(qtype, srcs)
    fg.run(scheduler=sched, max_passes=kw.pop("max_passes", 200000), **kw)
    out = []
    for i in range(len(srcs)):
        try:
            out.append(fg.fetch(i))
        except fork.ForkError as e:  # earlier waves keep digests only
            assert e.code == fork.FORK_E_STATE
            out.append(np.full(g.num_vertices, -1, np.int32))
    out = np.stack(out)
    st = fg.stats()
    fg.close()
    return out, st


def test_hand_fixture_all_sources_tiny_partitions():
    fork = _fork()
    nv, edges, expect = load_sp_fixture("sssp_bfs_hand8.txt")
    s, d, w = zip(*edges)
    g = fi.from_edges(nv, s, d, w)
    for pv in (1, 2, 8):
        say("hand fixture pv", pv)
        got, _ = run_sp(fork, g, np.arange(nv), "sssp", partition_vertices=pv)
        np.testing.assert_array_equal(got, oracle.sssp(g, np.arange(nv)))
        got, _ = run_sp(fork, g, np.arange(nv), "bfs", partition_vertices=pv)
        np.testing.assert_array_equal(got, oracle.bfs(g, np.arange(nv)))
        for (kind, src), vec in expect.items():
            ref = oracle.sssp(g, [src])[0] if kind == "sssp" else oracle.bfs(g, [src])[0]
            np.testing.assert_array_equal(ref, vec)


@pytest.mark.parametrize("seed", range(4))
def test_random_small_graphs(seed):
    fork = _fork()
    n = [10, 64, 200, 700][seed]
    g = fi.random_small(n, 4 * n, 40 + seed, wmax=[3, 50, 255, 1000][seed])
    srcs = np.arange(min(n, 48))
    for pv in (4, 64):
        say("random small", seed, "pv", pv)
        got, _ = run_sp(fork, g, srcs, "sssp", partition_vertices=pv)
        np.testing.assert_array_equal(got, oracle.sssp(g, srcs))
        got, _ = run_sp(fork, g, srcs, "bfs", partition_vertices=pv)
        np.testing.assert_array_equal(got, oracle.bfs(g, srcs))


@pytest.mark.parametrize("sched", ["priority", "fifo", "random", "maxops"])
def test_rmat12_sssp64_bit_exact(sched):
    """R-MAT scale 12, 64 SSSP queries: bit-exact under every schedule."""
    fork = _fork()
    spec = fi.WORKLOADS["rmat12_sssp64"]
    g = fi.make_graph(spec)
    srcs = fi.make_sources(g, spec)[0][1]
    say("rmat12", sched)
    got, st = run_sp(fork, g, srcs, "sssp", sched=sched)
    ref = oracle.sssp(g, srcs)
    np.testing.assert_array_equal(got, ref)
    for i in range(0, 64, 16):
        assert oracle.sp_certificate(g, srcs[i], got[i]) == 0
    assert st["passes"] > 0 and st["edges"] > 0


def test_rmat12_tiny_partition_stress():
    """Partitions of 1..16 vertices exercise the cross-partition machinery."""
    fork = _fork()
    spec = fi.WORKLOADS["rmat12_sssp64"]
    g = fi.make_graph(spec)
    srcs = fi.make_sources(g, spec)[0][1][:16]
    ref = oracle.sssp(g, srcs)
    for pv in (1, 16):
        say("tiny partitions", pv)
        got, st = run_sp(fork, g, srcs, "sssp", partition_vertices=pv)
        np.testing.assert_array_equal(got, ref)


def test_grid_sssp_bfs_mixed_batch():
    fork = _fork()
    g = fi.grid(96, 80, weights=(1, 1000), weight_seed=7)
    s1 = fi.sources_uniform(g, 24, 1)
    s2 = fi.sources_uniform(g, 24, 2)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=640)
    fg.submit("sssp", s1)
    fg.submit("bfs", s2)
    say("grid mixed")
    fg.run(max_passes=500000)
    d = np.stack([fg.fetch(i) for i in range(24)])
    lv = np.stack([fg.fetch(24 + i) for i in range(24)])
    np.testing.assert_array_equal(d, oracle.sssp(g, s1))
    np.testing.assert_array_equal(lv, oracle.bfs(g, s2))
    fg.close()


def check_ppr(g, srcs, P, R, eps, mode=0, tol=1e-4):
    for i, s in enumerate(srcs):
        p = P[i].astype(np.float64)
        r = R[i].astype(np.float64)
        assert np.all(p >= 0) and np.all(r >= 0)
        assert oracle.push_terminal(g, R[i], eps, mode, dtype=np.float32), f"query {i}: not terminal"
        inv = oracle.ppr_invariant_l1(g, s, p, r, ALPHA)
        assert inv <= tol, f"query {i}: invariant L1 {inv}"


@pytest.mark.parametrize("mode", [0, 1])
def test_ppr_small_invariant(mode):
    fork = _fork()
    g = fi.rmat(10, seed=12)
    srcs = fi.sources_uniform(g, 32, 3)
    eps = 1e-6 if mode == 0 else 1e-7
    for pv in (16, 128):
        say("ppr small mode", mode, "pv", pv)
        fg = fork.ForkGraph.from_graph(g, partition_vertices=pv)
        fg.submit("ppr", srcs, alpha=ALPHA, epsilon=eps, eps_mode=mode)
        fg.run(max_passes=200000)
        P = np.stack([fg.fetch(i, fork.FIELD_P) for i in range(len(srcs))])
        R = np.stack([fg.fetch(i, fork.FIELD_R) for i in range(len(srcs))])
        fg.close()
        check_ppr(g, srcs, P, R, eps, mode)


def test_pool_exhaustion_splits_waves():
    """A pool too small for all queries at once: the run splits the wave, every
    query's digest matches the oracle and the resident vectors are exact."""
    fork = _fork()
    spec = fi.WORKLOADS["rmat12_sssp64"]
    g = fi.make_graph(spec)
    srcs = fi.make_sources(g, spec)[0][1]
    say("small pool")
    fg = fork.ForkGraph.from_graph(g, partition_vertices=256, pool_bytes=1 << 22)
    fg.submit("sssp", srcs)
    fg.run(max_passes=200000)
    st = fg.stats()
    ref = oracle.sssp(g, srcs)
    resident = 0
    for i in range(len(srcs)):
        d = fg.digest(i)
        assert (d["count"], d["sum"], d["hash"]) == sp_digest(ref[i]), i
        try:
            np.testing.assert_array_equal(fg.fetch(i), ref[i])
            resident += 1
        except fork.ForkError as e:
            assert e.code == fork.FORK_E_STATE
    fg.close()
    assert resident >= 1
    say("waves", st["waves"])


def test_explicit_waves_digests():
    """max_queries forces waves; digests of all waves match the oracle."""
    fork = _fork()
    g = fi.rmat(11, seed=5, weights=(1, 255), weight_seed=6)
    srcs = fi.sources_uniform(g, 40, 8)
    fg = fork.ForkGraph.from_graph(g, max_queries=16)
    fg.submit("bfs", srcs[:20])
    fg.submit("sssp", srcs[20:])
    fg.run(max_passes=200000)
    st = fg.stats()
    assert st["waves"] == 3
    ref = np.concatenate([oracle.bfs(g, srcs[:20]), oracle.sssp(g, srcs[20:])])
    for i in range(40):
        d = fg.digest(i)
        assert (d["count"], d["sum"], d["hash"]) == sp_digest(ref[i]), i
    for i in range(32, 40):
        np.testing.assert_array_equal(fg.fetch(i), ref[i])
    with pytest.raises(fork.ForkError):
        fg.fetch(0)
    fg.close()


@pytest.mark.parametrize("sched", ["priority", "fifo"])
def test_persistent_kernel_parity(sched):
    """The persistent cooperative kernel gives the same exact SSSP/BFS results
    and valid PPR results as the per-pass kernels."""
    fork = _fork()
    g = fi.rmat(12, seed=1, weights=(1, 255), weight_seed=101)
    s1 = fi.sources_uniform(g, 24, 4)
    s2 = fi.sources_uniform(g, 16, 5)
    s3 = fi.sources_uniform(g, 16, 6)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=512)
    fg.submit("sssp", s1)
    fg.submit("bfs", s2)
    fg.submit("ppr", s3, alpha=ALPHA, epsilon=1e-6, eps_mode=1)
    say("persistent", sched)
    fg.run(scheduler=sched, persistent=1, max_passes=100000)
    d = np.stack([fg.fetch(i) for i in range(24)])
    lv = np.stack([fg.fetch(24 + i) for i in range(16)])
    np.testing.assert_array_equal(d, oracle.sssp(g, s1))
    np.testing.assert_array_equal(lv, oracle.bfs(g, s2))
    P = np.stack([fg.fetch(40 + i, fork.FIELD_P) for i in range(16)])
    R = np.stack([fg.fetch(40 + i, fork.FIELD_R) for i in range(16)])
    st = fg.stats()
    fg.close()
    check_ppr(g, s3, P, R, 1e-6, 1)
    assert st["passes"] > 1


def test_persistent_grid():
    fork = _fork()
    g = fi.grid(128, 96, weights=(1, 1000), weight_seed=9)
    s1 = fi.sources_uniform(g, 32, 11)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=1024)
    fg.submit("sssp", s1)
    say("persistent grid")
    fg.run(persistent=1, max_passes=1000000)
    d = np.stack([fg.fetch(i) for i in range(32)])
    fg.close()
    np.testing.assert_array_equal(d, oracle.sssp(g, s1))


@pytest.mark.parametrize("slots,persistent", [(256, 0), (1024, 0), (256, 1)])
def test_hashed_slice_parity(slots, persistent):
    """Hashed LDS slice: the visit keeps only touched vertices in an LDS hash
    table; with 256 slots and 4096-vertex partitions many vertices find no
    slot and are updated in global memory, so both paths are exercised."""
    fork = _fork()
    g = fi.rmat(13, seed=2, weights=(1, 255), weight_seed=102)
    s1 = fi.sources_uniform(g, 24, 14)
    s2 = fi.sources_uniform(g, 16, 15)
    s3 = fi.sources_uniform(g, 16, 16)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=4096)
    fg.submit("sssp", s1)
    fg.submit("bfs", s2)
    fg.submit("ppr", s3, alpha=ALPHA, epsilon=1e-6, eps_mode=1)
    say("hashed slice", slots, "persistent", persistent)
    fg.run(slice_slots=slots, persistent=persistent, max_passes=200000)
    d = np.stack([fg.fetch(i) for i in range(24)])
    lv = np.stack([fg.fetch(24 + i) for i in range(16)])
    np.testing.assert_array_equal(d, oracle.sssp(g, s1))
    np.testing.assert_array_equal(lv, oracle.bfs(g, s2))
    P = np.stack([fg.fetch(40 + i, fork.FIELD_P) for i in range(16)])
    R = np.stack([fg.fetch(40 + i, fork.FIELD_R) for i in range(16)])
    fg.close()
    check_ppr(g, s3, P, R, 1e-6, 1)


def test_hashed_slice_grid_and_bad_slots():
    fork = _fork()
    g = fi.grid(128, 96, weights=(1, 1000), weight_seed=19)
    s1 = fi.sources_uniform(g, 32, 21)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=4096)
    fg.submit("sssp", s1)
    with pytest.raises(fork.ForkError) as e:
        fg.run(slice_slots=300)                         # not a multiple of 256
    assert e.value.code == fork.FORK_E_INVALID
    say("hashed slice grid")
    fg.run(slice_slots=512, max_passes=1000000)
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(32)]), oracle.sssp(g, s1))
    fg.run(slice_slots=768, max_passes=1000000)          # a table size that is not a power of two
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(32)]), oracle.sssp(g, s1))
    fg.run(slice_slots=0, max_passes=1000000)           # back to the dense slice in the same context
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(32)]), oracle.sssp(g, s1))
    fg.close()


def test_large_partitions_use_hashed_slice():
    """Partitions of 32K-64K vertices do not fit a dense LDS slice: the library
    picks a hashed slice by itself, and explicit slot counts work too.  On a
    grid a visit's frontier is a narrow wavefront, so these runs stay below the
    frontier-spill bound."""
    fork = _fork()
    g = fi.grid(256, 512, weights=(1, 1000), weight_seed=23)
    s1 = fi.sources_uniform(g, 12, 17)
    s3 = fi.sources_uniform(g, 8, 18)
    ref = oracle.sssp(g, s1)
    for pv, slots in ((65536, 0), (32768, 2048), (65536, 8192)):
        say("large partitions", pv, slots)
        fg = fork.ForkGraph.from_graph(g, partition_vertices=pv)
        fg.submit("sssp", s1)
        fg.submit("ppr", s3, alpha=ALPHA, epsilon=1e-6, eps_mode=1)
        fg.run(slice_slots=slots, max_passes=200000)
        assert fg.stats()["spill_max"] <= 32768
        np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(12)]), ref)
        P = np.stack([fg.fetch(12 + i, fork.FIELD_P) for i in range(8)])
        R = np.stack([fg.fetch(12 + i, fork.FIELD_R) for i in range(8)])
        fg.close()
        check_ppr(g, s3, P, R, 1e-6, 1)


def test_large_rmat_partitions_stop_at_the_spill_bound():
    """On R-MAT 17 a visit of a 32K-64K-vertex partition activates far more
    vertices than its frontier holds: measured at 36,600-72,400 retained per
    visit, above the bound of 32,768.  That regime stops with FORK_E_CAPACITY
    and says why; the batch then runs at 16,384-vertex partitions (about
    10,800 retained) with exact distances."""
    fork = _fork()
    g = fi.rmat(17, seed=3, weights=(1, 255), weight_seed=103)
    s1 = fi.sources_uniform(g, 12, 17)
    s3 = fi.sources_uniform(g, 8, 18)
    say("rmat17 65536-vertex partitions, expecting the spill refusal")
    fg = fork.ForkGraph.from_graph(g, partition_vertices=65536)
    fg.submit("sssp", s1)
    fg.submit("ppr", s3, alpha=ALPHA, epsilon=1e-6, eps_mode=1)
    with pytest.raises(fork.ForkError) as e:
        fg.run(max_passes=200000)
    assert e.value.code == fork.FORK_E_CAPACITY and "frontier-spill" in str(e.value)
    fg.close()
    say("rmat17 16384-vertex partitions")
    fg = fork.ForkGraph.from_graph(g, partition_vertices=16384)
    fg.submit("sssp", s1)
    fg.submit("ppr", s3, alpha=ALPHA, epsilon=1e-6, eps_mode=1)
    fg.run(max_passes=200000)
    assert 0 < fg.stats()["spill_max"] <= 32768
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(12)]), oracle.sssp(g, s1))
    P = np.stack([fg.fetch(12 + i, fork.FIELD_P) for i in range(8)])
    R = np.stack([fg.fetch(12 + i, fork.FIELD_R) for i in range(8)])
    fg.close()
    check_ppr(g, s3, P, R, 1e-6, 1)


def test_four_byte_weights_and_clamped_tentative_sums():
    """Weights above 65535 use the 4-byte weight path; a non-shortest path whose
    length exceeds INT32_MAX is clamped while the true distance is exact."""
    fork = _fork()
    rng = np.random.default_rng(40)
    n, m = 300, 1500
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    w = rng.integers(1 << 21, 1 << 22, m)
    # a separate triangle: n -> n+1 -> n+2 costs 3e9 (beyond int32), n -> n+2 costs 2e9
    src = np.concatenate([src, [n, n + 1, n]])
    dst = np.concatenate([dst, [n + 1, n + 2, n + 2]])
    w = np.concatenate([w, [1_500_000_000, 1_500_000_000, 2_000_000_000]])
    g = fi.from_edges(n + 3, src, dst, w)
    srcs = np.asarray([n, 5, 17, 123], np.uint32)
    ref = oracle.sssp(g, srcs)
    assert ref[0, n + 2] == 2_000_000_000 and ref[0, n + 1] == 1_500_000_000
    for pv in (16, 4096):
        say("4-byte weights pv", pv)
        out, _ = run_sp(fork, g, srcs, partition_vertices=pv)
        np.testing.assert_array_equal(out, ref)


def test_degenerate_sources_and_repeated_sources():
    """Sources without out-edges (isolated or dangling), the same source
    submitted several times, and one source run as SSSP, BFS and PPR."""
    fork = _fork()
    g = fi.rmat(12, seed=41, weights=(1, 255), weight_seed=141)
    deg = g.out_degree()
    indeg = np.bincount(g.col, minlength=g.num_vertices)
    isolated = np.flatnonzero((deg == 0) & (indeg == 0))[:3]
    dangling = np.flatnonzero((deg == 0) & (indeg > 0))[:3]
    hub = int(np.argmax(deg))
    srcs = np.concatenate([isolated, dangling, [hub, hub, 7, 7]]).astype(np.uint32)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=256)
    fg.submit("sssp", srcs)
    fg.submit("bfs", srcs)
    fg.submit("ppr", srcs, alpha=ALPHA, epsilon=1e-6, eps_mode=1)
    say("degenerate sources", srcs.tolist())
    fg.run(max_passes=200000)
    n = len(srcs)
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(n)]), oracle.sssp(g, srcs))
    np.testing.assert_array_equal(np.stack([fg.fetch(n + i) for i in range(n)]), oracle.bfs(g, srcs))
    P = np.stack([fg.fetch(2 * n + i, fork.FIELD_P) for i in range(n)])
    R = np.stack([fg.fetch(2 * n + i, fork.FIELD_R) for i in range(n)])
    fg.close()
    check_ppr(g, srcs, P, R, 1e-6, 1)
    for i in range(len(isolated) + len(dangling)):
        # no out-edges: all mass stops at the source (p = alpha, the rest leaks)
        assert P[i, srcs[i]] == pytest.approx(ALPHA, rel=1e-6) and P[i].sum() == pytest.approx(ALPHA, rel=1e-6)


def test_one_partition_and_one_query_per_wave():
    """The whole graph in one partition (every edge stays inside it), and waves
    of a single query each (every wave re-initialises state and buffers)."""
    fork = _fork()
    g = fi.rmat(11, seed=42, weights=(1, 99), weight_seed=142)
    srcs = fi.sources_uniform(g, 6, 43)
    ref = oracle.sssp(g, srcs)
    say("one partition")
    out, st = run_sp(fork, g, srcs, partition_vertices=1 << 12)
    assert st["num_partitions"] == 1
    np.testing.assert_array_equal(out, ref)
    say("one query per wave")
    fg = fork.ForkGraph.from_graph(g, partition_vertices=128, max_queries=1)
    fg.submit("sssp", srcs)
    fg.run(max_passes=200000)
    assert fg.stats()["waves"] == len(srcs)
    for i in range(len(srcs)):
        assert (fg.digest(i)["count"], fg.digest(i)["sum"], fg.digest(i)["hash"]) == sp_digest(ref[i])
    np.testing.assert_array_equal(fg.fetch(len(srcs) - 1), ref[-1])  # the last wave stays resident
    fg.close()
