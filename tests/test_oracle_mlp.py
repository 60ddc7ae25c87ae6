"""Pins of the FP64 emulator reference: gradients against central finite
differences, GELU against its closed form at known points, and Adam against
its first-step closed form."""
import math

import numpy as np

from oracle import mlp


def test_gelu_known_values():
    z = np.array([0.0, 1.0, -1.0, 3.0])
    # x Phi(x): Phi(1) = 0.841344746..., Phi(3) = 0.998650102...
    np.testing.assert_allclose(mlp.gelu(z), [0.0, 0.8413447460685429, -0.15865525393145707, 3 * 0.9986501019683699]
                               , rtol=1e-12, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), rtol=1e-8)


def test_gradients_match_finite_differences():
    sizes = (6, 9, 7, 5, 8)  # small widths, same structure
    W, b = mlp.init(seed=3, sizes=sizes)
    rng = np.random.default_rng(0)
    x = rng.normal(size=(11, 6))
    t = rng.normal(size=(11, 8))
    gW, gb = mlp.grads(W, b, x, t)
    h = 1e-6
    for l in range(len(W)):
        for (i, j) in [(0, 0), (W[l].shape[0] - 1, W[l].shape[1] - 1), (1, 2)]:
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (mlp.loss(Wp, b, x, t) - mlp.loss(Wm, b, x, t)) / (2 * h)
            assert abs(fd - gW[l][i, j]) <= 1e-6 * max(1.0, abs(fd)), (l, i, j)
        for i in [0, b[l].shape[0] - 1]:
            bp = [v.copy() for v in b]
            bm = [v.copy() for v in b]
            bp[l][i] += h
            bm[l][i] -= h
            fd = (mlp.loss(W, bp, x, t) - mlp.loss(W, bm, x, t)) / (2 * h)
            assert abs(fd - gb[l][i]) <= 1e-6 * max(1.0, abs(fd)), (l, i)


def test_adam_first_step_closed_form():
    # after one step with zero moments the update is lr * g / (|g| + eps)
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -0.01, 0.0])]
    opt = mlp.Adam(p, [], lr=0.1)
    opt.m, opt.v = [np.zeros(3)], [np.zeros(3)]
    out = opt.step(p, g)[0]
    np.testing.assert_allclose(out, p[0] - 0.1 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    sizes = (6, 32, 32, 32, 8)
    W, b = mlp.init(seed=1, sizes=sizes)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(64, 6))
    t = np.tanh(x @ rng.normal(size=(6, 8)))
    opt = mlp.Adam(W, b, lr=3e-3)
    l0 = mlp.loss(W, b, x, t)
    for _ in range(200):
        gW, gb = mlp.grads(W, b, x, t)
        new = opt.step(W + b, gW + gb)
        W, b = new[:4], new[4:]
    assert mlp.loss(W, b, x, t) < 0.2 * l0
