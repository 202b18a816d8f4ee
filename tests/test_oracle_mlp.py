"""Pins of the FP64 surrogate-network reference (oracle/mlp.py), CPU only.

Each check is fixed by something other than the code under test: central
finite differences of the loss (the gradient), weights for which the network
reduces to a closed form (the forward pass), the first Adam step from zero
moments (-lr g / (|g| + eps) exactly), and the descent of the loss.
"""
import numpy as np
import pytest

from oracle import mlp as OM


def rand_problem(seed=0, n=37):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.4, OM.N_PARAMS)
    X = rng.uniform(-1, 1, (n, 3))
    T = rng.normal(0, 1, (n, 3))
    M = (rng.uniform(0, 1, (n, 3)) > 0.2).astype(float)
    return theta, X, T, M


def test_parameter_count_and_layout():
    assert OM.N_PARAMS == 64 * 3 + 64 + 64 * 64 + 64 + 3 * 64 + 3 == 4611
    theta = np.arange(OM.N_PARAMS, dtype=float)
    p = OM.unpack(theta)
    assert p["W1"][1, 0] == 3 and p["b1"][0] == 192 and p["W2"][0, 1] == 257
    assert p["b3"][2] == OM.N_PARAMS - 1
    assert np.array_equal(OM.pack(p), theta)


def test_gradient_matches_central_differences():
    theta, X, T, M = rand_problem()
    L, g = OM.loss_and_grad(theta, X, T, M)
    assert L == pytest.approx(OM.loss(theta, X, T, M), rel=1e-15)
    rng = np.random.default_rng(1)
    # every bias and a sample of every weight block
    idx = np.concatenate([np.arange(192, 256), np.arange(4352, 4416), np.arange(4608, 4611),
                          rng.choice(192, 20, replace=False), 256 + rng.choice(4096, 60, replace=False),
                          4416 + rng.choice(192, 20, replace=False)])
    # h = 1e-5: truncation error ~h^2 times the third derivative and rounding
    # ~1e-16 L / h, both far below the 1e-9 absolute / 1e-6 relative bar; a
    # dropped term or a wrong
    # sign or index changes the gradient at order one
    h = 1e-5
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (OM.loss(theta + e, X, T, M) - OM.loss(theta - e, X, T, M)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_forward_reduces_to_closed_forms():
    X = np.random.default_rng(2).uniform(-1, 1, (5, 3))
    # zero weights: the output is b3 and the hidden layers are tanh(b)
    p = {name: np.zeros(shape) for name, shape in OM.SHAPES}
    p["b3"] = np.array([0.5, -1.0, 2.0])
    y, (h1, h2) = OM.forward(OM.pack(p), X)
    assert np.allclose(y, p["b3"]) and np.all(h1 == 0) and np.all(h2 == 0)
    # one path: x0 -> unit 0 -> unit 0 -> output 1, weights a, b, c
    a, b, c = 0.7, -1.3, 2.5
    p["W1"][0, 0], p["W2"][0, 0], p["W3"][1, 0] = a, b, c
    y, _ = OM.forward(OM.pack(p), X)
    assert np.allclose(y[:, 1], -1.0 + c * np.tanh(b * np.tanh(a * X[:, 0])), atol=1e-15)
    assert np.allclose(y[:, 0], 0.5) and np.allclose(y[:, 2], 2.0)


def test_masked_entries_do_not_contribute():
    theta, X, T, M = rand_problem(3)
    T2 = T.copy()
    T2[M == 0] += 100.0  # garbage where masked
    L1, g1 = OM.loss_and_grad(theta, X, T, M)
    L2, g2 = OM.loss_and_grad(theta, X, T2, M)
    assert L1 == L2 and np.array_equal(g1, g2)


def test_first_adam_step_is_normalised_gradient():
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = OM.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, lr, 0.9, 0.999, eps)
    assert np.allclose(th1, theta - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_the_loss_on_a_smooth_target():
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (64, 3))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1], X[:, 1] * X[:, 2], np.cos(X[:, 2])], axis=1)
    theta = rng.normal(0, 0.3, OM.N_PARAMS)
    th, losses = OM.train(theta, X, T, np.ones_like(T), 300, 1e-2)
    assert losses[-1] < 0.05 * losses[0]
