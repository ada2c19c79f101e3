"""Rank-predictor MLP, forward / backward / Adam in FP64 (oracle side).

Not from the paper: the paper picks an anticipated ID rank l from its
observed rank-growth laws before compressing (Section 4, the paragraph on
cost evaluation). Here a small network predicts, per separator, the largest
ID rank of its HSS compression so that the sample count l = k^ + p_os can
be set before the compression runs.

Network: 8 -> 64 -> 64 -> 1, tanh on the two hidden layers, linear output;
target log2(1 + k); loss = mean squared error over the batch.
Weights are row-major [out, in]; biases [out].
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
      w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

SIZES = (8, 64, 64, 1)


def init_params(seed: int = 0):
    rng = np.random.default_rng(seed)
    params = []
    for i in range(3):
        fan_in, fan_out = SIZES[i], SIZES[i + 1]
        W = rng.standard_normal((fan_out, fan_in)) / np.sqrt(fan_in)
        b = np.zeros(fan_out)
        params += [W, b]
    return params


def forward(params, X):
    """X: [n, 8] -> (prediction [n], cache)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    a1 = np.tanh(z1)
    z2 = a1 @ W2.T + b2
    a2 = np.tanh(z2)
    y = a2 @ W3.T + b3
    return y[:, 0], (X, a1, a2)


def loss_and_grad(params, X, t):
    """MSE loss 1/n sum (y - t)^2 and its gradient w.r.t. every parameter."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, a1, a2) = forward(params, X)
    n = X.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = (2.0 / n) * r[:, None]              # [n, 1]
    gW3 = dy.T @ a2
    gb3 = dy.sum(axis=0)
    da2 = dy @ W3
    dz2 = da2 * (1.0 - a2 * a2)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    da1 = dz2 @ W2
    dz1 = da1 * (1.0 - a1 * a1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    if not state:
        state["t"] = 0
        state["m"] = [np.zeros_like(p) for p in params]
        state["v"] = [np.zeros_like(p) for p in params]
    state["t"] += 1
    t = state["t"]
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        state["m"][i] = b1 * state["m"][i] + (1 - b1) * g
        state["v"][i] = b2 * state["v"][i] + (1 - b2) * g * g
        mh = state["m"][i] / (1 - b1 ** t)
        vh = state["v"][i] / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out


def train(X, t, steps=500, lr=1e-2, seed=0):
    params = init_params(seed)
    state: dict = {}
    losses = []
    for _ in range(steps):
        loss, g = loss_and_grad(params, X, t)
        losses.append(loss)
        params = adam_step(params, g, state, lr=lr)
    return params, losses
