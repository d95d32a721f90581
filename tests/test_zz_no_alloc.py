"""The allocation-free training entry point (fork_mlp_train_noalloc, for
callers that cannot allocate) against fork_mlp_train on the same inputs: two
calls in a row, the second with fewer samples, so that the shared scratch
array's leftovers from the first call must not leak into the second."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _fork():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_14915_amd as fork
    return fork


def _close(a, b, steps, lr):
    # the same kernels and batches; only the order of the gradient's atomic
    # sums differs, which can flip the sign of a near-zero gradient entry and
    # so move that coordinate by a few lr over the steps (Adam's step is ~lr)
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    assert np.mean(d <= 1e-6 + 1e-5 * np.abs(a)) >= 0.995, np.sort(d)[-10:]
    assert np.all(d <= 4 * steps * lr), np.sort(d)[-10:]


def test_no_alloc_training_matches_fork_mlp_train():
    fork = _fork()
    import torch
    rng = np.random.default_rng(21)
    theta0 = omlp.init(13).astype(np.float32)
    for n, steps, batch, lr, seed in ((3000, 7, 256, 3e-3, 5), (500, 4, 128, 1e-3, 6)):
        x = rng.normal(size=(n, 16)).astype(np.float32)
        t = (x[:, 0] - np.abs(x[:, 1])).astype(np.float32)
        ref, ref_loss = fork.mlp_train(theta0, x, t, steps=steps, batch=batch, lr=lr, seed=seed)
        th = torch.from_numpy(theta0.copy()).cuda()
        xt = torch.from_numpy(x).cuda()
        tt = torch.from_numpy(t).cuda()
        lt = torch.full((steps,), 123.0, dtype=torch.float32, device="cuda")
        fork.mlp_train_noalloc(th, xt, tt, steps=steps, batch=batch, lr=lr, seed=seed, losses=lt)
        torch.cuda.synchronize()
        got = th.cpu().numpy()
        np.testing.assert_allclose(lt.cpu().numpy(), ref_loss, rtol=1e-4, atol=1e-6)
        _close(got, ref, steps, lr)


def test_no_alloc_training_rejects_too_many_samples():
    fork = _fork()
    import torch
    n = 32769
    th = torch.zeros(fork.MLP_NPARAM, dtype=torch.float32, device="cuda")
    xt = torch.zeros((n, 16), dtype=torch.float32, device="cuda")
    tt = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(fork.ForkError) as e:
        fork.mlp_train_noalloc(th, xt, tt, steps=1)
    assert e.value.code == fork.FORK_E_INVALID and "32768" in str(e.value)
