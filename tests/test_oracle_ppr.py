"""Pins for the oracle's PPR (CPU only): dense linear solve, closed forms on a
directed cycle and a chain, mass conservation, and the forward-push invariant.
"""
import numpy as np
import pytest

import fpp_inputs as fi
import oracle

ALPHA = 0.15


def dense_ppr(g, s, alpha):
    """pi = alpha (I - (1-alpha) P^T)^{-1} e_s with P = D^-1 A (zero rows for dangling)."""
    n = g.num_vertices
    A = np.zeros((n, n))
    src = np.repeat(np.arange(n), g.out_degree())
    np.add.at(A, (src, g.col.astype(np.int64)), 1.0)
    deg = A.sum(1)
    P = np.divide(A, deg[:, None], out=np.zeros_like(A), where=deg[:, None] > 0)
    e = np.zeros(n)
    e[s] = 1.0
    return alpha * np.linalg.solve(np.eye(n) - (1 - alpha) * P.T, e)


@pytest.mark.parametrize("seed", range(8))
def test_power_iteration_vs_dense_solve(seed):
    n = [2, 7, 30, 64, 100, 128, 200, 256][seed]
    g = fi.random_small(n, 2 * n + 3, 500 + seed, weighted=False)
    srcs = np.arange(min(n, 5))
    pi = oracle.ppr_exact(g, srcs, ALPHA)
    for i, s in enumerate(srcs):
        np.testing.assert_allclose(pi[i], dense_ppr(g, s, ALPHA), rtol=0, atol=1e-12)


def test_cycle_closed_form():
    # directed cycle of length n: pi_s(s+k) = alpha (1-alpha)^k / (1 - (1-alpha)^n)
    n = 13
    g = fi.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    pi = oracle.ppr_exact(g, [4], ALPHA)[0]
    k = (np.arange(n) - 4) % n
    ref = ALPHA * (1 - ALPHA) ** k / (1 - (1 - ALPHA) ** n)
    np.testing.assert_allclose(pi, ref, rtol=1e-13, atol=0)
    assert abs(pi.sum() - 1.0) < 1e-13


def test_chain_leaks_at_dangling_end():
    # s -> t with t dangling: pi(s) = alpha, pi(t) = alpha (1-alpha); total 1 - (1-alpha)^2
    g = fi.from_edges(2, [0], [1])
    pi = oracle.ppr_exact(g, [0], ALPHA)[0]
    np.testing.assert_allclose(pi, [ALPHA, ALPHA * (1 - ALPHA)], rtol=1e-14)
    # parallel edges count with multiplicity: 0->1 twice, 0->2 once
    g = fi.from_edges(3, [0, 0, 0], [1, 1, 2])
    pi = oracle.ppr_exact(g, [0], ALPHA)[0]
    np.testing.assert_allclose(pi, [ALPHA, ALPHA * (1 - ALPHA) * 2 / 3, ALPHA * (1 - ALPHA) / 3],
                               rtol=1e-14)


def test_mass_is_one_without_dangling():
    rng = np.random.default_rng(3)
    n = 50
    src = np.concatenate([np.arange(n), rng.integers(0, n, 100)])
    dst = np.concatenate([(np.arange(n) + 1) % n, rng.integers(0, n, 100)])
    g = fi.from_edges(n, src, dst)
    pi = oracle.ppr_exact(g, [0, 17], ALPHA)
    np.testing.assert_allclose(pi.sum(1), 1.0, atol=1e-12)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_forward_push_invariant_and_termination(seed, mode):
    n = [20, 64, 128, 256][seed]
    g = fi.random_small(n, 4 * n, 900 + seed, weighted=False)
    eps = 1e-4
    srcs = np.arange(3)
    p, r = oracle.forward_push(g, srcs, ALPHA, eps, mode)
    for i, s in enumerate(srcs):
        pi = dense_ppr(g, s, ALPHA)
        # push invariant: p + PPR(r) = PPR(e_s)
        pr = np.zeros(n)
        for u in np.flatnonzero(r[i]):
            pr += r[i][u] * dense_ppr(g, u, ALPHA)
        np.testing.assert_allclose(p[i] + pr, pi, atol=1e-12)
        assert oracle.ppr_invariant_l1(g, s, p[i], r[i], ALPHA) < 1e-12
        assert oracle.push_terminal(g, r[i], eps, mode)
        assert np.all(p[i] >= 0) and np.all(r[i] >= 0)
        # error bound: ||pi - p||_1 = ||PPR(r)||_1 <= ||r||_1
        assert np.abs(pi - p[i]).sum() <= r[i].sum() + 1e-12


def test_push_converges_as_eps_shrinks():
    g = fi.rmat(9, seed=4)
    s = fi.sources_uniform(g, 1, 5)
    pi = oracle.ppr_exact(g, s, ALPHA)[0]
    errs = []
    for eps in (1e-3, 1e-5, 1e-7, 1e-9):
        p, r = oracle.forward_push(g, s, ALPHA, eps)
        errs.append(np.abs(pi - p[0]).sum())
        assert errs[-1] <= r[0].sum() + 1e-12
    assert errs == sorted(errs, reverse=True) and errs[-1] < 1e-5


def test_invariant_detects_planted_mistake():
    g = fi.random_small(40, 160, 77, weighted=False)
    p, r = oracle.forward_push(g, [0], ALPHA, 1e-5)
    assert oracle.ppr_invariant_l1(g, 0, p[0], r[0], ALPHA) < 1e-12
    bad = p[0].copy()
    v = int(np.argmax(bad))
    bad[v] *= 1.001  # a 0.1% error at one vertex
    assert oracle.ppr_invariant_l1(g, 0, bad, r[0], ALPHA) > 1e-5
    # residual that was dropped instead of pushed (mass lost) is detected too
    r_bad = r[0].copy()
    r_bad[np.argmax(r_bad)] = 0.0
    assert oracle.ppr_invariant_l1(g, 0, p[0], r_bad, ALPHA) > 1e-7


def test_push_terminal_fp32_threshold_decision():
    """The GPU keeps r in fp32 and decides a push with thr = fp32(eps) (mode 0)
    or fp32(eps) * fp32(outdeg) (mode 1) in fp32; push_terminal(dtype=float32)
    takes the same decision.  A residual planted exactly at the fp32
    threshold is active; one fp32 ulp below it is not."""
    # vertex 0 has out-degree 3, vertex 1 out-degree 1, vertex 2 none
    g = fi.from_edges(3, [0, 0, 0, 1], [1, 2, 2, 0])
    eps = 1e-6  # not representable in fp32: fp32(eps) < eps
    e32 = np.float32(eps)
    assert float(e32) < eps
    for mode in (0, 1):
        for v in (0, 1, 2):
            d = int(g.out_degree()[v])
            thr32 = np.float32(e32 * np.float32(d)) if mode else e32
            if mode and d == 0:
                continue  # threshold 0: any positive residual is active
            r = np.zeros(3, np.float32)
            r[v] = thr32
            assert not oracle.push_terminal(g, r, eps, mode, dtype=np.float32), (mode, v)
            r[v] = np.nextafter(thr32, np.float32(0))
            assert oracle.push_terminal(g, r, eps, mode, dtype=np.float32), (mode, v)
    # the fp64 decision differs exactly here: fp32(eps) is below eps in fp64
    r = np.zeros(3, np.float32)
    r[1] = e32
    assert oracle.push_terminal(g, r, eps, 0, dtype=np.float64)
    assert not oracle.push_terminal(g, r, eps, 0, dtype=np.float32)
    # a dangling vertex in mode 1 has threshold 0: any positive residual is active
    r = np.zeros(3, np.float32)
    r[2] = np.float32(1e-30)
    assert not oracle.push_terminal(g, r, eps, 1, dtype=np.float32)
    r[2] = 0.0
    assert oracle.push_terminal(g, r, eps, 1, dtype=np.float32)
