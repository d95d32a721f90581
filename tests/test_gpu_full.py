"""GPU parity at the workloads' full graph sizes, plus the error paths of the
C ABI on a real device.

Full-size runs use the autotuned knobs of the workload (as bench.py does)
and check the outputs the CPU oracle can compute one by one: a seeded sample
of queries compared element by element (SSSP/BFS bit-exact, PPR push
invariant within 1e-4 L1 and termination), plus the optimality certificate
and digests.  The scale-22 and scale-23 graphs run a seeded subset of their
queries (the full query sets take minutes of GPU time)."""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle
from digests import sp_digest

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


# knobs autotuned for the scale-20 R-MAT SSSP+PPR mix; used for R-MAT graphs without a cached tuning
RMAT_KNOBS = {"partition_vertices": 16384, "items_per_pass": 16384, "window": 16, "delta": 512, "persistent": 0,
              "slice_slots": 0}


def knobs(g, queries, fallback=None):
    from paper_2103_14915_amd import autotune
    return autotune.cached(g, queries) or dict(fallback or autotune.DEFAULTS)


def run_workload(fork, g, queries, spec, p):
    """The workload as bench.py runs it: tuned knobs and the workload's vertex order."""
    from paper_2103_14915_amd import order
    fg = fork.ForkGraph.from_graph(g, partition_vertices=p["partition_vertices"],
                                   vertex_order=order.auto(spec, g, p["partition_vertices"]))
    for qt, s in queries:
        fg.submit(qt, s, alpha=spec.get("alpha", 0.15), epsilon=spec.get("epsilon", 1e-6),
                  eps_mode=spec.get("eps_mode", 0))
    from paper_2103_14915_amd import autotune
    fg.run(**autotune.run_kwargs(p))
    return fg


def check_sp_sample(fork, fg, g, srcs, first_id, kind, n, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(srcs), min(n, len(srcs)), replace=False))
    ref = oracle.sssp(g, srcs[idx]) if kind == "sssp" else oracle.bfs(g, srcs[idx])
    resident = 0
    for k, i in enumerate(idx):
        d = fg.digest(first_id + int(i))  # digests exist for every wave
        assert (d["count"], d["sum"], d["hash"]) == sp_digest(ref[k]), f"{kind} query {i} digest"
        try:
            got = fg.fetch(first_id + int(i))
        except fork.ForkError as e:  # vectors stay resident for the last wave only
            assert e.code == fork.FORK_E_STATE
            continue
        resident += 1
        np.testing.assert_array_equal(got, ref[k], err_msg=f"{kind} query {i}")
        assert oracle.sp_certificate(g, srcs[i], got, unit_weights=kind == "bfs") == 0
    return resident


def check_ppr_sample(fork, fg, g, srcs, first_id, spec, n, seed):
    rng = np.random.default_rng(seed)
    eps, mode, alpha = spec["epsilon"], spec.get("eps_mode", 0), spec["alpha"]
    idx = np.sort(rng.choice(len(srcs), min(n, len(srcs)), replace=False))
    keep = []
    for i in idx:  # vectors of earlier waves are not resident; their digests are checked
        d = fg.digest(first_id + int(i))
        assert d["fsum"] > 0.14 and d["fres"] >= 0.0 and d["fsum"] + d["fres"] <= 1.0 + 1e-3
        try:
            fg.fetch(first_id + int(i), fork.FIELD_P)
            keep.append(i)
        except fork.ForkError as e:
            assert e.code == fork.FORK_E_STATE
    idx = np.asarray(keep, np.int64)
    if idx.size == 0:
        return
    P = np.stack([fg.fetch(first_id + int(i), fork.FIELD_P) for i in idx]).astype(np.float64)
    R32 = np.stack([fg.fetch(first_id + int(i), fork.FIELD_R) for i in idx])
    R = R32.astype(np.float64)
    x0 = -R.copy()
    x0[np.arange(len(idx)), srcs[idx].astype(np.int64)] += 1.0
    ref = oracle.ppr_power(g, x0, alpha)
    for k, i in enumerate(idx):
        assert np.all(P[k] >= 0) and np.all(R[k] >= 0)
        assert oracle.push_terminal(g, R32[k], eps, mode, dtype=np.float32), f"ppr query {i}"
        inv = float(np.abs(P[k] - ref[k]).sum())
        assert inv <= 1e-4, f"ppr query {i}: invariant L1 {inv}"


def test_error_paths_on_device():
    fork = _fork()
    g = fi.rmat(10, seed=3, weights=(1, 9), weight_seed=4)
    fg = fork.ForkGraph.from_graph(g)
    with pytest.raises(fork.ForkError) as e:
        fg.run()
    assert e.value.code == fork.FORK_E_STATE            # nothing submitted
    fg.submit("sssp", [1, 2, 3])
    with pytest.raises(fork.ForkError) as e:
        fg.fetch(0)
    assert e.value.code == fork.FORK_E_STATE            # not run yet
    with pytest.raises(fork.ForkError) as e:
        fg.submit("sssp", [5, g.num_vertices])          # one bad source: nothing enqueued
    assert e.value.code == fork.FORK_E_INVALID
    with pytest.raises(fork.ForkError) as e:
        fg.submit("ppr", [5], alpha=1.5)
    assert e.value.code == fork.FORK_E_INVALID
    with pytest.raises(fork.ForkError) as e:
        fg.submit(7, [5])
    assert e.value.code == fork.FORK_E_INVALID
    fg.run()
    assert fg.stats()["waves"] == 1
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(3)]), oracle.sssp(g, [1, 2, 3]))
    with pytest.raises(fork.ForkError) as e:
        fg.fetch(0, fork.FIELD_P)                       # SSSP has no p vector
    assert e.value.code == fork.FORK_E_INVALID
    with pytest.raises(fork.ForkError) as e:
        fg.fetch(3)
    assert e.value.code == fork.FORK_E_INVALID
    with pytest.raises(fork.ForkError) as e:
        fg.run(max_passes=1)                            # far fewer passes than needed
    assert e.value.code == fork.FORK_E_NOT_CONVERGED
    fg.run()                                            # the context stays usable
    np.testing.assert_array_equal(fg.fetch(2), oracle.sssp(g, [3])[0])
    fg.close()


def test_rmat20_ppr4096_full():
    fork = _fork()
    spec = fi.WORKLOADS["rmat20_ppr4096"]
    g = fi.make_graph(spec)
    queries = fi.make_sources(g, spec)
    p = knobs(g, queries)
    say("rmat20 ppr4096", p)
    fg = run_workload(fork, g, queries, spec, p)
    srcs = queries[0][1]
    d = [fg.digest(i) for i in range(len(srcs))]
    assert all(x["fsum"] > 0.14 and x["fres"] >= 0 for x in d)
    check_ppr_sample(fork, fg, g, srcs, 0, spec, 8, 1)
    # sweep cuts of every resident query (the NCP application), a sample against the oracle
    import time
    from oracle import ncp
    fg.sweep(0, 4)  # builds the reverse adjacency
    t0 = time.perf_counter()
    res = fg.sweep(0, len(srcs), 1024)
    say("sweep of", len(srcs), "queries:", round((time.perf_counter() - t0) * 1e3, 1), "ms")
    assert all(r["flags"] == 0 and r["swept"] == min(r["support"], 1024) for r in res)
    for i in np.random.default_rng(5).choice(len(srcs), 3, replace=False):
        p = fg.fetch(int(i), fork.FIELD_P)
        order, cut, vol, phi = ncp.sweep_profile(g, p, 1024)
        k, best = ncp.best_cut(phi)
        r = res[int(i)]
        assert (r["best_size"], r["best_cut"], r["best_volume"]) == (k, int(cut[k - 1]), int(vol[k - 1]))
        assert r["best_conductance"] == best
    fg.close()


@pytest.mark.skip(reason="one run of this case (65,536-vertex partitions, before certified queries were limited "
                  "to partitions of at most 1,024 vertices) ended in a GPU memory fault whose cause is not found; "
                  "it stays off the GPU until that cause is found")
def test_rmat20_ppr_certified_sample():
    """The scale-20 PPR workload's graph and sources (the first 64), run in
    the L1-certified mode: every query ends with ||r||_1 <= 0.9e-4, and a
    seeded sample is within 1e-4 of fp64 power iteration in L1."""
    fork = _fork()
    spec = fi.WORKLOADS["rmat20_ppr4096"]
    g = fi.make_graph(spec)
    queries = fi.make_sources(g, spec)
    p = knobs(g, queries)
    srcs = queries[0][1][:64]
    say("rmat20 certified ppr64", p)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=p["partition_vertices"])
    fg.submit("ppr", srcs, alpha=spec["alpha"], epsilon=spec["epsilon"], eps_mode=spec["eps_mode"], l1_target=1e-4)
    fg.run(items_per_pass=p["items_per_pass"], window=p["window"], delta=p["delta"],
           slice_slots=p.get("slice_slots", 0))
    st = fg.stats()
    say("refine rounds", st["refine_rounds"], "edges", st["edges"], "run_ms", round(st["run_ms"], 1))
    assert st["refine_rounds"] >= 1
    for i in range(len(srcs)):
        d = fg.digest(i)
        assert 0.0 <= d["fres"] <= 0.9e-4 * (1 + 1e-6), (i, d["fres"])
    idx = np.sort(np.random.default_rng(7).choice(len(srcs), 4, replace=False))
    P = np.stack([fg.fetch(int(i), fork.FIELD_P) for i in idx]).astype(np.float64)
    fg.close()
    pi = oracle.ppr_exact(g, srcs[idx], spec["alpha"])
    for k, i in enumerate(idx):
        err = float(np.abs(P[k] - pi[k]).sum())
        say("query", int(i), "L1 to power iteration", err)
        assert np.all(P[k] >= 0) and err <= 1e-4, (int(i), err)


def test_rmat20_ppr_certified_on_frontier_sized_partitions():
    """The scale-20 PPR workload's graph and its first 32 sources in the
    L1-certified mode, on 1,024-vertex partitions (the largest the certified
    mode accepts, so a refinement never overflows a visit's frontier): every
    query ends with ||r||_1 <= 0.9e-4, no visit retains more activated
    vertices than its partition holds, and a seeded sample of 4 queries is
    within 1e-4 of fp64 power iteration in L1, never above it."""
    fork = _fork()
    spec = fi.WORKLOADS["rmat20_ppr4096"]
    g = fi.make_graph(spec)
    queries = fi.make_sources(g, spec)
    srcs = queries[0][1][:32]
    say("rmat20 certified ppr32 on 1024-vertex partitions")
    fg = fork.ForkGraph.from_graph(g, partition_vertices=1024)
    fg.submit("ppr", srcs, alpha=spec["alpha"], epsilon=spec["epsilon"], eps_mode=spec["eps_mode"], l1_target=1e-4)
    fg.run(engine="buffered")
    st = fg.stats()
    say("refine rounds", st["refine_rounds"], "edges", st["edges"], "spill_max", st["spill_max"],
        "run_ms", round(st["run_ms"], 1))
    assert st["refine_rounds"] >= 1 and st["spill_max"] <= 1024
    for i in range(len(srcs)):
        d = fg.digest(i)
        assert 0.0 <= d["fres"] <= 0.9e-4 * (1 + 1e-6), (i, d["fres"])
    idx = np.sort(np.random.default_rng(7).choice(len(srcs), 4, replace=False))
    P = np.stack([fg.fetch(int(i), fork.FIELD_P) for i in idx]).astype(np.float64)
    R = np.stack([fg.fetch(int(i), fork.FIELD_R) for i in idx]).astype(np.float64)
    fg.close()
    pi = oracle.ppr_exact(g, srcs[idx], spec["alpha"])
    for k, i in enumerate(idx):
        err = float(np.abs(P[k] - pi[k]).sum())
        say("query", int(i), "L1 to power iteration", err, "||r||_1", float(R[k].sum()))
        assert np.all(P[k] >= 0) and err <= 1e-4, (int(i), err)
        assert err <= R[k].sum() + 1e-5, (int(i), err, float(R[k].sum()))


def test_grid2048_sssp_bfs_full():
    fork = _fork()
    spec = fi.WORKLOADS["grid2048_sssp1024_bfs1024"]
    g = fi.make_graph(spec)
    queries = fi.make_sources(g, spec)
    p = knobs(g, queries)
    say("grid2048", p)
    fg = run_workload(fork, g, queries, spec, p)
    check_sp_sample(fork, fg, g, queries[0][1], 0, "sssp", 12, 2)
    check_sp_sample(fork, fg, g, queries[1][1], 1024, "bfs", 12, 3)
    # every query reaches the whole (connected) grid
    assert all(fg.digest(i)["count"] == g.num_vertices for i in range(0, 2048, 97))
    fg.close()


@pytest.mark.parametrize("name,take", [("rmat22_mixed16384", (256, 128, 128)),
                                       ("rmat23_sssp_ppr65536", (128, 128))])
def test_large_rmat_query_subset(name, take):
    """Full-size scale-22 / scale-23 graphs with a seeded subset of the queries."""
    fork = _fork()
    spec = fi.WORKLOADS[name]
    g = fi.make_graph(spec)
    queries = [(qt, s[:k]) for (qt, s), k in zip(fi.make_sources(g, spec), take)]
    p = knobs(g, queries, RMAT_KNOBS)
    say(name, [len(s) for _, s in queries], p)
    fg = run_workload(fork, g, queries, spec, p)
    first = 0
    for k, (qt, s) in enumerate(queries):
        if qt == "ppr":
            check_ppr_sample(fork, fg, g, s, first, spec, 4, 10 + k)
        else:
            check_sp_sample(fork, fg, g, s, first, qt, 6, 10 + k)
        first += len(s)
    fg.close()


@pytest.mark.parametrize("name,take", [("rmat20_sssp_ppr2048", 1024), ("rmat23_sssp_ppr65536", 1024)])
def test_sssp_ppr_mix_in_the_bench_configuration(name, take):
    """The SSSP+PPR batches on the knobs bench.py takes for them: the scale-20
    mix in full, and a seeded 2,048-query slice of the scale-23 batch on the
    knobs tuned on a subset of it (the grouped engine for both).  Sampled SSSP
    distances are bit-exact against Dijkstra; sampled PPR vectors meet the push
    gates and the invariant against power iteration."""
    fork = _fork()
    spec = fi.WORKLOADS[name]
    g = fi.make_graph(spec)
    full = fi.make_sources(g, spec)
    p = knobs(g, full)
    assert p.get("engine") == "grouped", p
    queries = [(qt, s[:take]) for qt, s in full]
    say(name, [len(s) for _, s in queries], p)
    fg = run_workload(fork, g, queries, spec, p)
    assert [qt for qt, _ in queries] == ["sssp", "ppr"]
    check_sp_sample(fork, fg, g, queries[0][1], 0, "sssp", 6, 31)
    check_ppr_sample(fork, fg, g, queries[1][1], take, spec, 4, 32)
    fg.close()


def test_rmat22_mixed_full_in_the_bench_configuration():
    """All 16,384 queries of the scale-22 mixed batch (8,192 SSSP, 4,096 BFS,
    4,096 PPR) on the knobs bench.py takes for it, tuned on a 512-per-type
    subset of the same graph; the batch runs in several waves.  A seeded
    sample per type is checked against the oracle: SSSP/BFS digests (and the
    vectors of the last, resident wave) bit-exact, PPR digests within the mass
    bounds and resident PPR vectors through the push gates."""
    fork = _fork()
    spec = fi.WORKLOADS["rmat22_mixed16384"]
    g = fi.make_graph(spec)
    queries = fi.make_sources(g, spec)
    p = knobs(g, queries)
    assert p.get("engine") == "grouped", p
    say("rmat22 mixed, all queries", [len(s) for _, s in queries], p)
    fg = run_workload(fork, g, queries, spec, p)
    st = fg.stats()
    say("waves", st["waves"], "passes", st["passes"])
    assert st["waves"] >= 2
    first = 0
    for k, (qt, s) in enumerate(queries):
        if qt == "ppr":
            check_ppr_sample(fork, fg, g, s, first, spec, 3, 50 + k)
        else:
            check_sp_sample(fork, fg, g, s, first, qt, 4, 50 + k)
        first += len(s)
    fg.close()


def test_rmat20_ppr_absolute_threshold_on_the_grouped_engine():
    """PPR forward push as the configuration states it: R-MAT 20, alpha 0.15,
    absolute threshold epsilon = 1e-6 (a vertex pushes while r(u) >= 1e-6),
    on a seeded 256-source subset of its 4,096 sources.  About 1.4e8 edge
    pushes per query, so the pushes of a group's 64 queries overlap on most
    vertices.  The grouped engine runs it (no operation pool).  Sampled
    vectors: every residual below epsilon, and p within L1 1e-4 of the
    fixpoint that the invariant p + PPR(r) = PPR(e_s) fixes (power iteration,
    fp64)."""
    fork = _fork()
    spec = fi.WORKLOADS["rmat20_ppr4096_abs"]
    assert spec["eps_mode"] == 0 and spec["epsilon"] == 1e-6
    g = fi.make_graph(spec)
    (qt, srcs), = fi.make_sources(g, spec)
    srcs = srcs[:256]
    p = dict(engine="grouped", partition_vertices=4096, items_per_pass=0, window=0, delta=0, mu=0.0, persistent=0,
             slice_slots=0, group_threads=1024)
    say("rmat20 ppr absolute", len(srcs), p)
    fg = run_workload(fork, g, [(qt, srcs)], spec, p)
    d = [fg.digest(i) for i in range(len(srcs))]
    # every query's mass: p sums to at least alpha (the source's first push), p and r to at most 1
    assert all(x["fsum"] > 0.14 and x["fres"] >= 0 and x["fsum"] + x["fres"] <= 1.0 + 1e-3 for x in d)
    check_ppr_sample(fork, fg, g, srcs, 0, spec, 4, 41)
    fg.close()
