"""Cost-model network reference — test infrastructure only (float64 NumPy).

The learned scheduler's network: 5 inputs -> 64 ReLU -> 64 ReLU -> 1, trained
by mean-squared error with Adam.  The GPU library keeps the parameters as one
float32 vector of 4,609 entries in this order:

  W1 [64 x 5] (row j holds the weights into hidden unit j), b1 [64],
  W2 [64 x 64] (row k: weights into second-layer unit k),   b2 [64],
  w3 [64], b3 [1].

This module writes the same network out in float64 so the GPU forward,
gradient and optimizer kernels can be compared with it; its own gradient is
checked against central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 5, 64
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("w3", (N_HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    assert theta.shape == (N_PARAMS,)
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[off:off + k].reshape(shape)
        off += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SIZES])


def forward(theta, X):
    """Predictions y[rows] for inputs X[rows, 5]."""
    P = unpack(theta)
    X = np.asarray(X, np.float64)
    h1 = np.maximum(X @ P["W1"].T + P["b1"], 0.0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0)
    return h2 @ P["w3"] + P["b3"][0]


def loss(theta, X, T):
    y = forward(theta, X)
    return float(np.mean((y - np.asarray(T, np.float64)) ** 2))


def loss_and_grad(theta, X, T):
    """L = mean over rows of (y - t)^2 and dL/dtheta (chain rule, layer by layer)."""
    P = unpack(theta)
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    B = X.shape[0]
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["w3"] + P["b3"][0]
    r = y - T
    L = float(np.mean(r ** 2))
    dy = 2.0 * r / B                      # dL/dy
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, P["w3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def adam_step(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015); `step` counts from 1."""
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v
