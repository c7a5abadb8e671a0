"""Float64 reference for the plan cost model: a 3-layer perceptron.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network (hidden width H, input width F):
    h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3
Loss over a batch of B rows with targets t (log run time):
    loss = (1/B) sum_i (y_i - t_i)^2
Gradients are the hand-derived chain rule below; Adam follows Kingma & Ba
(bias-corrected first and second moments).  Parameters are a dict of arrays
W1 (H,F), b1 (H,), W2 (H,H), b2 (H,), W3 (1,H), b3 (1,).
"""

from __future__ import annotations

import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(params, X):
    X = np.asarray(X, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], dtype=np.float64) for k in NAMES)
    z1 = X @ W1.T + b1
    h1 = np.tanh(z1)
    z2 = h1 @ W2.T + b2
    h2 = np.tanh(z2)
    y = h2 @ W3.T + b3
    return y[:, 0], (X, h1, h2)


def loss(params, X, t) -> float:
    y, _ = forward(params, X)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean((y - t) ** 2))


def backward(params, X, t):
    """Gradients of the mean squared error with respect to every parameter."""
    W2 = np.asarray(params["W2"], dtype=np.float64)
    W3 = np.asarray(params["W3"], dtype=np.float64)
    y, (X, h1, h2) = forward(params, X)
    t = np.asarray(t, dtype=np.float64)
    B = X.shape[0]
    dy = 2.0 * (y - t) / B                # (B,)
    gW3 = dy[None, :] @ h2                # (1,H)
    gb3 = np.array([dy.sum()])
    dh2 = dy[:, None] * W3                # (B,H)
    dz2 = dh2 * (1.0 - h2 * h2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (1.0 - h1 * h1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3}


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; ``state`` holds m, v (dicts) and step t."""
    state["t"] = state.get("t", 0) + 1
    tt = state["t"]
    for k in NAMES:
        g = np.asarray(grads[k], dtype=np.float64)
        m = state.setdefault("m", {}).setdefault(k, np.zeros_like(g))
        v = state.setdefault("v", {}).setdefault(k, np.zeros_like(g))
        m[...] = beta1 * m + (1.0 - beta1) * g
        v[...] = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** tt)
        vhat = v / (1.0 - beta2 ** tt)
        params[k] = np.asarray(params[k], dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return params


def train(params, X, t, steps, lr=1e-3):
    state = {}
    p = {k: np.array(v, dtype=np.float64) for k, v in params.items()}
    for _ in range(steps):
        adam_step(p, backward(p, X, t), state, lr=lr)
    return p
