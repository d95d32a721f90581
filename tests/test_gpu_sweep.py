"""GPU sweep cuts (fork_sweep) against the oracle's sweep of the same PPR
vectors.  The PPR vectors themselves are checked by the push invariant in the
parity tests; here the oracle (oracle/ncp.py) sweeps the vector the GPU
returned, with the same internal positions, and every reported figure must
match exactly: support, prefixes swept, best size, cut, volume and
conductance (fp64 quotients of integers), and the per-size minima."""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
from oracle import ncp

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


def check(g, p, res, max_size, pos=None):
    order, cut, vol, phi = ncp.sweep_profile(g, p, max_size, pos)
    support = ncp.sweep_order(g, p, None, pos).size
    assert res["flags"] == 0
    assert res["support"] == support and res["swept"] == order.size
    k, best = ncp.best_cut(phi)
    assert res["best_size"] == k
    if k:
        assert res["best_conductance"] == best
        assert (res["best_cut"], res["best_volume"]) == (int(cut[k - 1]), int(vol[k - 1]))
    else:
        assert np.isinf(res["best_conductance"])
    mins = ncp.ncp([phi], max_size)
    got = np.asarray(res["size_min"])
    np.testing.assert_array_equal(got[:mins.size], mins)
    assert np.all(np.isinf(got[mins.size:]))


@pytest.mark.parametrize("scale,eps,max_size,ordered", [(10, 1e-5, 1024, False), (10, 1e-5, 37, False),
                                                        (10, 1e-5, 1, False), (12, 1e-7, 1024, False),
                                                        (12, 1e-7, 700, True)])
def test_sweep_matches_the_oracle(scale, eps, max_size, ordered):
    fork = _fork()
    g = fi.rmat(scale, seed=81)
    srcs = fi.sources_uniform(g, 12, 82)
    pos = np.random.default_rng(83).permutation(g.num_vertices).astype(np.uint32) if ordered else None
    say("sweep scale", scale, "eps", eps, "max_size", max_size, "ordered", ordered)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=256, vertex_order=pos)
    fg.submit("ppr", srcs, alpha=ALPHA, epsilon=eps, eps_mode=0)
    fg.run(max_passes=400000)
    res = fg.sweep(0, len(srcs), max_size)
    P = [fg.fetch(i, fork.FIELD_P) for i in range(len(srcs))]
    fg.close()
    big = 0
    for i in range(len(srcs)):
        check(g, P[i], res[i], max_size, pos)
        big += res[i]["support"] > max_size
    if scale == 12:
        assert big > 0  # the radix-select path ran


def test_two_cliques_sweep_finds_the_seed_clique():
    fork = _fork()
    m = 20
    s, t = [], []
    for base in (0, m):
        for i in range(m):
            for j in range(m):
                if i != j:
                    s.append(base + i)
                    t.append(base + j)
    s += [0, m]
    t += [m, 0]
    g = fi.from_edges(2 * m, s, t)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=8)
    fg.submit("ppr", [3], alpha=ALPHA, epsilon=1e-8, eps_mode=0)
    fg.run(max_passes=400000)
    (res,) = fg.sweep(0, 1, 64)
    p = fg.fetch(0, fork.FIELD_P)
    fg.close()
    check(g, p, res, 64)
    assert res["best_size"] == m and res["best_cut"] == 2


def test_sweep_errors():
    fork = _fork()
    g = fi.rmat(9, seed=84)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=128, max_queries=4)
    a = fg.submit("sssp", [1, 2])
    b = fg.submit("ppr", fi.sources_uniform(g, 8, 85), alpha=ALPHA, epsilon=1e-5)
    with pytest.raises(fork.ForkError) as e:
        fg.sweep(b, 1)  # not run yet
    assert e.value.code == fork.FORK_E_STATE
    fg.run(max_passes=200000)
    for args, code in (((a, 1), fork.FORK_E_INVALID), ((b, 1, 0), fork.FORK_E_INVALID),
                       ((b, 1, 1025), fork.FORK_E_INVALID), ((b, 100), fork.FORK_E_INVALID),
                       ((b, 1), fork.FORK_E_STATE)):  # the first PPR queries ran in an earlier wave
        with pytest.raises(fork.ForkError) as e:
            fg.sweep(*args)
        assert e.value.code == code, args
    last = len(fg.types) - 1
    assert fg.sweep(last, 1)[0]["swept"] >= 1
    assert fg.sweep(last, 0) == []
    fg.close()
