"""Float64 reference of the mask-placement MLP -- TEST INFRASTRUCTURE ONLY.

12 -> 64 -> 64 -> 1 multilayer perceptron with ReLU, mean-squared-error loss
and Adam (Kingma & Ba, 2015). Parameters live in one flat vector in the
order W1 [64,12], b1 [64], W2 [64,64], b2 [64], W3 [64], b3 [1] (5,057
values), the layout the HIP kernels use. Everything is written out with
plain numpy matrix products so it can be checked by eye.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 12, 64
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)) and zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS)
    q = unpack(p)
    q["W1"][...] = rng.normal(0.0, np.sqrt(2.0 / N_IN), (N_H, N_IN))
    q["W2"][...] = rng.normal(0.0, np.sqrt(2.0 / N_H), (N_H, N_H))
    q["W3"][...] = rng.normal(0.0, np.sqrt(2.0 / N_H), (N_H,))
    return p


def forward(p, x):
    """x [B, 12] -> (y [B], cache)."""
    q = unpack(np.asarray(p, np.float64))
    x = np.asarray(x, np.float64)
    z1 = x @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ q["W3"] + q["b3"][0]
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t):
    y, _ = forward(p, x)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(p, x, t):
    """Analytic gradient of the mean-squared error, same flat layout as p."""
    q = unpack(np.asarray(p, np.float64))
    y, (x, z1, h1, z2, h2) = forward(p, x)
    B = x.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B
    g = np.zeros(N_PARAMS)
    G = unpack(g)
    G["W3"][...] = h2.T @ dy
    G["b3"][...] = dy.sum()
    dz2 = np.outer(dy, q["W3"]) * (z2 > 0)
    G["W2"][...] = dz2.T @ h1
    G["b2"][...] = dz2.sum(0)
    dz1 = (dz2 @ q["W2"]) * (z1 > 0)
    G["W1"][...] = dz1.T @ x
    G["b1"][...] = dz1.sum(0)
    return g


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
