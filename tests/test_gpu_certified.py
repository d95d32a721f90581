"""GPU parity of the L1-certified PPR mode against the fp64 oracle.

A forward push that stops at threshold eps leaves residual mass ||r||_1, and
by the push invariant (p + PPR(r) = PPR(e_s)) its estimate p is exactly
||PPR(r)||_1 <= ||r||_1 away from the PPR vector in L1.  With l1_target set,
the run keeps lowering the query's threshold until ||r||_1 <= 0.9 * target.
These tests check the result directly: ||p - pi_s||_1 <= target against
oracle power iteration, with pi_s itself pinned by the oracle's own tests.
"""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle

pytestmark = pytest.mark.gpu

ALPHA = 0.15
TARGET = 1e-4


def _fork():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_14915_amd as fork
    return fork


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fetch_pr(fork, fg, ids):
    P = np.stack([fg.fetch(i, fork.FIELD_P) for i in ids])
    R = np.stack([fg.fetch(i, fork.FIELD_R) for i in ids])
    return P, R


def check_certified(g, srcs, P, R, target=TARGET):
    pi = oracle.ppr_exact(g, srcs, ALPHA)
    for i, s in enumerate(srcs):
        p = P[i].astype(np.float64)
        r = R[i].astype(np.float64)
        assert np.all(p >= 0) and np.all(r >= 0)
        assert r.sum() <= 0.9 * target * (1 + 1e-6), f"query {i}: ||r||_1 = {r.sum()}"
        err = float(np.abs(p - pi[i]).sum())
        assert err <= target, f"query {i}: ||p - pi||_1 = {err}"
        # the estimate is short of pi by what r still carries: never above it
        assert err <= r.sum() + 1e-5, (err, r.sum())


@pytest.mark.parametrize("mode,eps,slots", [(0, 1e-6, 0), (1, 1e-6, 0), (1, 1e-6, 256)])
def test_certified_ppr_meets_l1_target(mode, eps, slots):
    fork = _fork()
    g = fi.rmat(12, seed=31)
    srcs = fi.sources_uniform(g, 24, 32)
    say("certified ppr mode", mode, "eps", eps, "slots", slots)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=512)
    fg.submit("ppr", srcs, alpha=ALPHA, epsilon=eps, eps_mode=mode, l1_target=TARGET)
    fg.run(max_passes=400000, slice_slots=slots)
    P, R = fetch_pr(fork, fg, range(len(srcs)))
    st = fg.stats()
    dg = [fg.digest(i) for i in range(len(srcs))]
    fg.close()
    assert st["refine_rounds"] >= 1  # eps alone leaves more than the target at this size
    check_certified(g, srcs, P, R)
    for i in range(len(srcs)):
        assert dg[i]["fres"] == pytest.approx(R[i].astype(np.float64).sum(), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("persistent", [0, 1])
def test_certified_ppr_in_a_mixed_batch(persistent):
    """SSSP, plain PPR and certified PPR in one wave: only the certified
    queries are refined; SSSP stays bit-exact and plain PPR stops at eps."""
    fork = _fork()
    g = fi.rmat(11, seed=41, weights=(1, 255), weight_seed=42)
    s_sp = fi.sources_uniform(g, 16, 43)
    s_pr = fi.sources_uniform(g, 12, 44)
    s_ce = fi.sources_uniform(g, 12, 45)
    eps = 1e-6
    say("certified mixed persistent", persistent)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=256)
    a = fg.submit("sssp", s_sp)
    b = fg.submit("ppr", s_pr, alpha=ALPHA, epsilon=eps, eps_mode=1)
    c = fg.submit("ppr", s_ce, alpha=ALPHA, epsilon=eps, eps_mode=1, l1_target=TARGET)
    fg.run(max_passes=400000, persistent=persistent)
    D = np.stack([fg.fetch(a + i) for i in range(len(s_sp))])
    Pb, Rb = fetch_pr(fork, fg, range(b, b + len(s_pr)))
    Pc, Rc = fetch_pr(fork, fg, range(c, c + len(s_ce)))
    st = fg.stats()
    fg.close()
    assert st["refine_rounds"] >= 1
    np.testing.assert_array_equal(D, oracle.sssp(g, s_sp))
    for i, s in enumerate(s_pr):
        assert oracle.push_terminal(g, Rb[i], eps, 1, dtype=np.float32)
        assert oracle.ppr_invariant_l1(g, s, Pb[i], Rb[i], ALPHA) <= 1e-4
    # the plain queries kept the mass eps leaves, far above the target
    assert np.median(Rb.astype(np.float64).sum(1)) > 10 * TARGET
    check_certified(g, s_ce, Pc, Rc)


def test_certified_target_already_met_needs_no_refinement():
    fork = _fork()
    g = fi.rmat(10, seed=51)
    srcs = fi.sources_uniform(g, 8, 52)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=128)
    fg.submit("ppr", srcs, alpha=ALPHA, epsilon=1e-6, eps_mode=0, l1_target=0.5)
    fg.run(max_passes=200000)
    P, R = fetch_pr(fork, fg, range(len(srcs)))
    st = fg.stats()
    fg.close()
    assert st["refine_rounds"] == 0
    for i in range(len(srcs)):
        assert oracle.push_terminal(g, R[i], 1e-6, 0, dtype=np.float32)
    check_certified(g, srcs, P, R, target=0.5)


def test_certified_needs_partitions_within_the_frontier():
    """Partitions larger than the visit's frontier (1,024 vertices) are
    refused before anything runs; the same queries run once the graph is
    loaded with smaller partitions."""
    fork = _fork()
    g = fi.rmat(12, seed=71)
    srcs = fi.sources_uniform(g, 4, 72)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=2048)
    fg.submit("ppr", srcs, alpha=ALPHA, epsilon=1e-6, eps_mode=1, l1_target=TARGET)
    with pytest.raises(fork.ForkError) as e:
        fg.run(max_passes=1000)
    assert e.value.code == fork.FORK_E_INVALID and "1024" in str(e.value)
    fg.close()
    fg = fork.ForkGraph.from_graph(g, partition_vertices=1024)
    fg.submit("ppr", srcs, alpha=ALPHA, epsilon=1e-6, eps_mode=1, l1_target=TARGET)
    fg.run(max_passes=400000)
    P, R = fetch_pr(fork, fg, range(len(srcs)))
    fg.close()
    check_certified(g, srcs, P, R)


def test_certified_bad_target_is_rejected():
    fork = _fork()
    g = fi.rmat(8, seed=61)
    fg = fork.ForkGraph.from_graph(g)
    for bad in (-1e-4, float("nan"), float("inf")):
        with pytest.raises(fork.ForkError) as e:
            fg.submit("ppr", [1, 2], alpha=ALPHA, epsilon=1e-6, l1_target=bad)
        assert e.value.code == fork.FORK_E_INVALID
    assert fg.submit("sssp", [3]) == 0  # nothing was enqueued by the failed calls
    fg.close()
