"""Pins of the cost-model network reference (float64): its gradient against
central finite differences, closed forms of the forward pass, and the first
Adam step (m and v start at zero, so the step is lr * g / (|g| + eps))."""
import numpy as np
import pytest

from oracle import mlp


def random_theta(seed, scale=0.5):
    return np.random.default_rng(seed).normal(0, scale, mlp.N_PARAMS)


def test_param_count():
    assert mlp.N_PARAMS == 5 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4609


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(100 + seed)
    theta = random_theta(seed)
    X = rng.normal(0, 1, (16, 5))
    T = rng.normal(0, 1, 16)
    _, g = mlp.loss_and_grad(theta, X, T)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    idx = np.concatenate([idx, [0, 319, 320, 383, 384, 4479, 4480, 4543, 4544, 4607, 4608]])
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss(theta + e, X, T) - mlp.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_forward_closed_forms():
    X = np.random.default_rng(3).normal(0, 1, (8, 5))
    theta = np.zeros(mlp.N_PARAMS)
    theta[-1] = 2.5                                   # only b3: constant output
    assert np.allclose(mlp.forward(theta, X), 2.5)
    P = mlp.unpack(random_theta(4))
    P["W1"][:] = 0
    P["b1"][:] = 1.0                                  # h1 = 1
    P["W2"][:] = 0
    P["W2"][:, 0] = 1.0
    P["b2"][:] = 0.0                                  # h2 = 1
    P["w3"][:] = 1.0
    P["b3"][:] = 0.0                                  # y = 64
    assert np.allclose(mlp.forward(mlp.pack(P), X), 64.0)
    P["b1"][:] = -1.0                                 # ReLU cuts everything: y = 0
    assert np.allclose(mlp.forward(mlp.pack(P), X), 0.0)


def test_first_adam_step():
    rng = np.random.default_rng(5)
    theta = rng.normal(0, 1, mlp.N_PARAMS)
    g = rng.normal(0, 1, mlp.N_PARAMS)
    new, m, v = mlp.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, lr=0.01)
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
