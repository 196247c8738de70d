"""Pins of the float64 MLP reference: finite-difference gradients, closed
forms, and Adam's first step."""
import numpy as np

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 5057


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) + rng.normal(0, 0.01, mlp.N_PARAMS)
    x = rng.normal(size=(37, 12))
    t = rng.normal(size=37)
    g = mlp.grad(p, x, t)
    h = 1e-6
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False), [mlp.N_PARAMS - 1]])
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss(p + e, x, t) - mlp.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_zero_weights_give_the_output_bias():
    p = np.zeros(mlp.N_PARAMS)
    p[-1] = 0.75
    y, _ = mlp.forward(p, np.random.default_rng(1).normal(size=(5, 12)))
    assert np.all(y == 0.75)


def test_single_path_closed_form():
    # one active path x0 -> h1_0 -> h2_0 -> y: y = w3 * relu(w2 * relu(w1 * x0))
    p = np.zeros(mlp.N_PARAMS)
    q = mlp.unpack(p)
    q["W1"][0, 0], q["W2"][0, 0], q["W3"][0] = 2.0, 3.0, 0.5
    x = np.array([[1.5] + [0.0] * 11, [-1.0] + [0.0] * 11])
    y, _ = mlp.forward(p, x)
    assert np.allclose(y, [0.5 * 3.0 * 2.0 * 1.5, 0.0])


def test_adam_first_step_moves_by_lr_times_sign():
    p = np.zeros(4)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p2, m, v = mlp.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # after bias correction the first step is lr * g / (|g| + eps)
    assert np.allclose(p2[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert p2[3] == 0.0
