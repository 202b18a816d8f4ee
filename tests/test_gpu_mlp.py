"""Surrogate-network kernels against the FP64 reference (needs an MI355X).

Forward pass, loss and gradient, and Adam training of the library's
3-64-64-3 network (include/lbm_mlp.h), called through the C ABI, against
oracle/mlp.py on the same seeded parameters and batches.

Tolerances (FP32 kernels vs FP64): every output and gradient entry is a sum
of at most 64 products per layer, accumulated over at most a few hundred
samples, so FP32 rounding (6e-8 relative) stays below ~1e-5 of the largest
magnitude involved; tanhf adds a few ulp.  The bars below are 2e-5 of the
largest output, 5e-5 of the largest gradient entry and 1e-5 relative in the
loss.  Adam divides by sqrt(v), so trajectories are compared after a few
steps on the loss and on the parameters that moved.
"""
import numpy as np
import pytest

from oracle import mlp as OM
from paper_1306_6445_amd import lbm

pytestmark = pytest.mark.gpu


def problem(seed, n, mask_frac=0.2):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.3, OM.N_PARAMS).astype(np.float32).astype(np.float64)
    X = rng.uniform(-1, 1, (n, 3)).astype(np.float32).astype(np.float64)
    T = rng.normal(0, 1, (n, 3)).astype(np.float32).astype(np.float64)
    M = (rng.uniform(0, 1, (n, 3)) > mask_frac).astype(np.float64)
    return theta, X, T, M


@pytest.mark.parametrize("n", [1, 31, 32, 100, 1000])
def test_forward_matches_oracle(n):
    theta, X, _, _ = problem(10 + n, n)
    with lbm.Mlp(theta, max_batch=1024) as net:
        y = net.forward(X)
    y64, _ = OM.forward(theta, X)
    assert np.abs(y - y64).max() <= 2e-5 * max(1.0, np.abs(y64).max())


@pytest.mark.parametrize("n", [1, 33, 77, 512])
def test_loss_and_gradient_match_oracle(n):
    theta, X, T, M = problem(20 + n, n)
    M[0, :] = 1.0  # at least one weighted entry
    with lbm.Mlp(theta, max_batch=512) as net:
        L, g = net.loss_grad(X, T, M)
    L64, g64 = OM.loss_and_grad(theta, X, T, M)
    assert L == pytest.approx(L64, rel=1e-5)
    assert np.abs(g - g64).max() <= 5e-5 * np.abs(g64).max()
    # every block of the parameter vector is produced (no stale slots)
    for name, sl in (("W1", slice(0, 192)), ("b1", slice(192, 256)), ("W2", slice(256, 4352)),
                     ("b2", slice(4352, 4416)), ("W3", slice(4416, 4608)), ("b3", slice(4608, 4611))):
        assert np.abs(g[sl] - g64[sl]).max() <= 5e-5 * np.abs(g64).max(), name


def test_adam_training_tracks_oracle():
    rng = np.random.default_rng(3)
    n = 200
    X = rng.uniform(-1, 1, (n, 3))
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1], X[:, 1] * X[:, 2], np.cos(X[:, 2] + X[:, 0])], axis=1)
    M = np.ones_like(T)
    theta0 = rng.normal(0, 0.3, OM.N_PARAMS).astype(np.float32).astype(np.float64)
    X = X.astype(np.float32).astype(np.float64)
    T = T.astype(np.float32).astype(np.float64)
    steps, lr = 10, 1e-3
    th64, losses = OM.train(theta0, X, T, M, steps, lr)
    with lbm.Mlp(theta0, max_batch=256) as net:
        last = net.train(X, T, M, steps, lr)
        assert net.steps_taken == steps
        th = net.params.astype(np.float64)
        L_after, _ = net.loss_grad(X, T, M)
    assert last == pytest.approx(losses[-1], rel=1e-4)
    assert L_after == pytest.approx(OM.loss(th64, X, T, M), rel=1e-4)
    # parameters: the moves (up to steps * lr) agree; Adam normalises each
    # gradient entry, so an entry whose gradient is within FP32 noise of zero
    # may step differently, and those are few
    d = np.abs(th - th64)
    assert np.median(d) < 1e-6
    assert np.mean(d > 0.1 * lr) < 0.01
    assert d.max() <= 2 * steps * lr


def test_training_continues_across_calls_and_reset():
    theta, X, T, M = problem(5, 64, 0.0)
    with lbm.Mlp(theta, max_batch=64) as net:
        net.train(X, T, M, 3, 1e-3)
        net.train(X, T, M, 2, 1e-3)
        th_split = net.params
        assert net.steps_taken == 5
        net.params = theta
        assert net.steps_taken == 0
        net.train(X, T, M, 5, 1e-3)
        assert np.array_equal(net.params, th_split)


def test_argument_errors():
    theta, X, T, M = problem(6, 40)
    with lbm.Mlp(theta, max_batch=32) as net:
        assert net.forward(X[:0]).shape == (0, 3)  # an empty batch is a no-op
        with pytest.raises(lbm.LbmError):
            net.loss_grad(X, T, M)  # 40 > max_batch
        with pytest.raises(lbm.LbmError):
            net.loss_grad(X[:8], T[:8], np.zeros((8, 3)))  # all weights zero
        with pytest.raises(lbm.LbmError):
            net.train(X[:8], T[:8], M[:8], 1, -1.0)
