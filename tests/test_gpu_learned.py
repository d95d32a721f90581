"""GPU tests of the learned scheduler: the MLP's forward and backward kernels
against the fp64 oracle, training on the GPU, trace capture, and exactness of
runs scheduled by the network."""
import sys

import numpy as np
import pytest

import fpp_inputs as fi
import oracle
from oracle import mlp as omlp

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


def test_mlp_forward_and_gradient_vs_fp64_oracle():
    fork = _fork()
    rng = np.random.default_rng(0)
    theta = (omlp.init(5) + rng.normal(0, 0.02, omlp.N_PARAMS)).astype(np.float32)
    for n in (1, 63, 64, 200):
        x = rng.normal(size=(n, 16)).astype(np.float32)
        t = rng.normal(size=n).astype(np.float32)
        y = fork.mlp_forward(theta, x)
        y64, _ = omlp.forward(theta.astype(np.float64), x.astype(np.float64))
        np.testing.assert_allclose(y, y64, rtol=1e-4, atol=1e-5)
        loss, g = fork.mlp_grad(theta, x, t)
        loss64, g64 = omlp.loss_and_grad(theta.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
        assert abs(loss - loss64) <= 1e-4 * max(1.0, abs(loss64))
        # relative error of the whole gradient vector, and per component where it is not tiny
        assert np.linalg.norm(g - g64) <= 1e-4 * np.linalg.norm(g64)
        big = np.abs(g64) > 1e-3 * np.abs(g64).max()
        np.testing.assert_allclose(g[big], g64[big], rtol=1e-3)


def test_mlp_training_on_gpu_reduces_loss():
    fork = _fork()
    rng = np.random.default_rng(1)
    x = rng.normal(size=(4096, 16)).astype(np.float32)
    t = (np.abs(x[:, 0]) - 0.5 * x[:, 1] + 0.25 * x[:, 2] * x[:, 3]).astype(np.float32)
    theta0 = omlp.init(3).astype(np.float32)
    l0 = omlp.loss_and_grad(theta0.astype(np.float64), x, t)[0]
    theta, losses = fork.mlp_train(theta0, x, t, steps=600, batch=256, lr=3e-3, seed=5)
    l1 = omlp.loss_and_grad(theta.astype(np.float64), x, t)[0]
    assert l1 < 0.2 * l0, (l0, l1)
    assert losses[-20:].mean() < losses[:20].mean()


def test_trace_and_learned_schedule_are_exact():
    """Trace a rule run, train on it, and run with the learned scores: SSSP and
    BFS stay bit-exact and PPR passes its gates."""
    fork = _fork()
    from paper_2103_14915_amd import learn
    g = fi.rmat(13, seed=31, weights=(1, 255), weight_seed=131)
    s_sp = fi.sources_mixed(g, 48, 7)
    s_pr = fi.sources_mixed(g, 16, 8)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=512)
    fg.submit("sssp", s_sp)
    fg.submit("ppr", s_pr, alpha=0.15, epsilon=1e-6, eps_mode=1)
    fg.run(scheduler="priority", trace=1)
    rec = fg.trace()
    say("trace records", rec.shape)
    assert rec.shape[0] > 10 and np.all(rec[:, 17] >= rec[:, 16]) and np.all(rec[:, 16] >= 0)
    ref = oracle.sssp(g, s_sp)
    np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(48)]), ref)
    theta, losses = learn.train(rec, steps=300, batch=64)
    assert np.isfinite(losses).all()
    for persistent in (0, 1):
        fg.run(scheduler="learned", mlp_weights=theta, persistent=persistent, max_passes=200000)
        np.testing.assert_array_equal(np.stack([fg.fetch(i) for i in range(48)]), ref)
        for i, s in enumerate(s_pr):
            p = fg.fetch(48 + i, fork.FIELD_P).astype(np.float64)
            r = fg.fetch(48 + i, fork.FIELD_R)
            assert oracle.push_terminal(g, r, 1e-6, 1, dtype=np.float32)
            assert oracle.ppr_invariant_l1(g, s, p, r.astype(np.float64), 0.15) <= 1e-4
    fg.close()


def test_learned_vs_rule_measured_on_the_same_queries():
    """What the committed network changes against the rule it replaces: both
    schedules run the same SSSP+PPR batch; SSSP results stay identical (and
    equal to the oracle), PPR passes its gates, and the ratio of the two
    run times is reported.  The network is not required to win here: the
    measured ratio on the scale-20 mix is documented with the design."""
    import time

    fork = _fork()
    from paper_2103_14915_amd import learn
    theta = np.load(learn.DEFAULT_WEIGHTS)
    g = fi.rmat(17, seed=33, weights=(1, 255), weight_seed=133)
    s_sp = fi.sources_mixed(g, 128, 34)
    s_pr = fi.sources_mixed(g, 64, 35)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=learn.PARTITION_VERTICES)
    fg.submit("sssp", s_sp)
    fg.submit("ppr", s_pr, alpha=0.15, epsilon=1e-6, eps_mode=1)
    kw = dict(learn.RUN_KW, max_passes=500000)
    ref = None
    best = {}
    for sched in ("priority", "learned", "priority", "learned"):
        t0 = time.perf_counter()
        fg.run(scheduler=sched, mlp_weights=theta if sched == "learned" else None, **kw)
        dt = time.perf_counter() - t0
        best[sched] = min(best.get(sched, dt), dt)
        d = np.stack([fg.fetch(i) for i in range(len(s_sp))])
        if ref is None:
            ref = d
            np.testing.assert_array_equal(d[:16], oracle.sssp(g, s_sp[:16]))
        np.testing.assert_array_equal(d, ref)
        for i in range(0, len(s_pr), 16):
            p = fg.fetch(len(s_sp) + i, fork.FIELD_P).astype(np.float64)
            r = fg.fetch(len(s_sp) + i, fork.FIELD_R)
            assert oracle.push_terminal(g, r, 1e-6, 1, dtype=np.float32)
            assert oracle.ppr_invariant_l1(g, s_pr[i], p, r.astype(np.float64), 0.15) <= 1e-4
    fg.close()
    ratio = best["priority"] / best["learned"]
    say(f"learned vs rule on R-MAT 17 (128 SSSP + 64 PPR): speedup {ratio:.3f} "
        f"(rule {best['priority'] * 1e3:.1f} ms, learned {best['learned'] * 1e3:.1f} ms)")
    assert ratio > 0.25  # no pathological slowdown


def test_learned_scheduler_gains_where_selection_binds():
    """Where the select step binds, the committed network's schedule beats the
    priority rule's in run time with identical SSSP results.  The workload is
    the scale-20 SSSP+PPR mix (R-MAT 20, 1,024 + 1,024 queries) on its tuned
    grouped-engine knobs with 512 work items per pass, so that each pass takes
    a few of the pending (partition, group) pairs.  Rule and learned runs
    alternate, nine of each (single runs vary by about 10%), and their medians
    are compared; on MI355X the gain measured 1.05-1.09x here (and 1.00x or
    below with 16 or 4 partitions per pass, where the test does not claim
    one)."""
    import statistics
    import time

    import torch

    fork = _fork()
    from paper_2103_14915_amd import autotune, learn
    spec = fi.WORKLOADS["rmat20_sssp_ppr2048"]
    g = fi.make_graph(spec)
    queries = fi.make_sources(g, spec)
    assert [qt for qt, _ in queries] == ["sssp", "ppr"]
    p = autotune.cached(g, queries)
    assert p and p["engine"] == "grouped", p
    theta = np.load(learn.DEFAULT_WEIGHTS)
    fg = fork.ForkGraph.from_graph(g, partition_vertices=p["partition_vertices"])
    for qt, s in queries:
        fg.submit(qt, s, alpha=spec["alpha"], epsilon=spec["epsilon"], eps_mode=spec["eps_mode"])
    kw = dict(autotune.run_kwargs(p), items_per_pass=512)
    fg.prepare(**kw)
    fg.run(**kw)  # warm-up
    nsp = len(queries[0][1])
    times = {"priority": [], "learned": []}
    ref = None
    for sched in ("priority", "learned") * 9:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fg.run(scheduler=sched, mlp_weights=theta if sched == "learned" else None, **kw)
        torch.cuda.synchronize()
        times[sched].append(time.perf_counter() - t0)
        dig = [(fg.digest(i)["hash"], fg.digest(i)["count"]) for i in range(nsp)]
        if ref is None:
            ref = dig
        assert dig == ref, f"{sched}: SSSP results differ"
    fg.close()
    speedup = statistics.median(times["priority"]) / statistics.median(times["learned"])
    say(f"learned vs rule, R-MAT 20 SSSP+PPR mix, 512 items per pass: speedup {speedup:.3f} "
        f"(rule {[round(t * 1e3) for t in times['priority']]} ms, learned {[round(t * 1e3) for t in times['learned']]} ms)")
    assert speedup > 1.0


@pytest.mark.parametrize("lr", [1e-3, 3e-2])
def test_adam_steps_on_gpu_match_the_fp64_oracle(lr):
    """Two fork_mlp_train steps with the whole sample set as the batch against
    oracle.mlp.adam_step fed with the fp64 gradient.  The batch is then the
    full set at every step, so the GPU's update is the oracle's up to fp32
    rounding of the gradient.  Where that rounding can flip a gradient's sign
    (|g| near zero) Adam's step is bounded by lr per step instead."""
    fork = _fork()
    rng = np.random.default_rng(11)
    n = 300
    x = rng.normal(size=(n, 16)).astype(np.float32)
    t = (x[:, 0] - 0.5 * np.abs(x[:, 1])).astype(np.float32)
    theta0 = (omlp.init(9) + rng.normal(0, 0.01, omlp.N_PARAMS)).astype(np.float32)
    th64 = theta0.astype(np.float64)
    m = np.zeros(omlp.N_PARAMS)
    v = np.zeros(omlp.N_PARAMS)
    gmin = np.full(omlp.N_PARAMS, np.inf)
    for step in (1, 2):
        _, g64 = omlp.loss_and_grad(th64, x.astype(np.float64), t.astype(np.float64))
        gmin = np.minimum(gmin, np.abs(g64))
        th64, m, v = omlp.adam_step(th64, g64, m, v, step, lr=lr)
        th_gpu, losses = fork.mlp_train(theta0, x, t, steps=step, batch=n, lr=lr, seed=3)
        say("adam step", step, "lr", lr, "loss", float(losses[-1]))
        sure = gmin > 1e-4  # gradient well above fp32 rounding at every step so far
        assert sure.sum() > 0.5 * omlp.N_PARAMS
        np.testing.assert_allclose(th_gpu[sure], th64[sure], rtol=0, atol=1e-5 * lr + 1e-6 * np.abs(th64[sure]).max())
        # Adam's bias-corrected step is at most about lr per coordinate: by
        # Cauchy-Schwarz |m^|/sqrt(v^) <= 1.0014 at t = 2 (and 1 at t = 1)
        assert np.all(np.abs(th_gpu.astype(np.float64) - theta0) <= step * lr * 1.0015 + 1e-7)
