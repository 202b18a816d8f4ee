"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

Only tests/, the package's smoke check and the benchmark's CPU leg may use this
module; the library's surrogate kernels never do.

Network (3 -> 64 -> 64 -> 3, tanh hidden units, linear output):
    h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3.
Loss over a batch with per-entry weights M (0 masks a missing target):
    L = sum_{i,k} M_ik (y_ik - t_ik)^2 / (2 sum_{i,k} M_ik).
Gradients by the chain rule written out layer by layer (no autodiff), and the
Adam update of Kingma & Ba (2015, Algorithm 1) with bias-corrected moments:
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parameter vector layout (row-major matrices, out x in):
    W1[64][3], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]   (4611 values).

Pins (tests/test_oracle_mlp.py): central finite differences of the loss,
special weights with closed-form outputs, Adam's first step equal to
-lr g / (|g| + eps), and the loss falling on a smooth target.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 3, 64, 3
SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, X):
    """Outputs y[n][3] and the hidden activations (h1, h2)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return y, (h1, h2)


def loss(theta, X, T, M) -> float:
    y, _ = forward(theta, X)
    M = np.asarray(M, dtype=np.float64)
    return float(np.sum(M * (y - T) ** 2) / (2.0 * np.sum(M)))


def loss_and_grad(theta, X, T, M):
    """(L, dL/dtheta) by backpropagation through the three layers."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    y, (h1, h2) = forward(theta, X)
    wsum = np.sum(M)
    L = float(np.sum(M * (y - T) ** 2) / (2.0 * wsum))
    dy = M * (y - T) / wsum                      # dL/dy
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dz2 = (dy @ p["W3"]) * (1.0 - h2 ** 2)       # through tanh: d tanh(z) = 1 - tanh(z)^2
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def adam_step(theta, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(theta, X, T, M, steps: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """Full-batch Adam for `steps` steps from zero moments; returns (theta, losses)."""
    theta = np.array(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for t in range(1, steps + 1):
        L, g = loss_and_grad(theta, X, T, M)
        losses.append(L)
        theta, m, v = adam_step(theta, m, v, g, t, lr, beta1, beta2, eps)
    return theta, np.array(losses)
