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


def test_bf16_rounding_matches_torch():
    # torch's float32 -> bfloat16 conversion rounds to nearest, ties to even
    import torch
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, size=4000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 1e-40, -1e-40, 1e-45]]).astype(np.float32)
    # exact ties: the 16 dropped bits are 0x8000, with even and odd kept parts
    u = rng.integers(0, 2 ** 31, size=1000, dtype=np.uint64).astype(np.uint32)
    ties = ((u & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)
    v = np.concatenate([v, ties[np.isfinite(ties)]])
    ref = torch.from_numpy(v.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(v), ref)


def test_bf16_mode_within_rounding_bound_of_exact():
    W, b = mlp.init(seed=4)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(40, 6))
    t = rng.normal(size=(40, 8))
    y = mlp.forward(W, b, x)
    yb = mlp.forward(W, b, x, rnd=mlp.bf16)
    u = 2.0 ** -9  # bf16 unit roundoff
    rel = np.linalg.norm(yb - y) / np.linalg.norm(y)
    assert 0 < rel < 8 * u
    gW, gb = mlp.grads(W, b, x, t)
    gWb, gbb = mlp.grads(W, b, x, t, rnd=mlp.bf16)
    for l in range(4):
        assert np.linalg.norm(gWb[l] - gW[l]) / np.linalg.norm(gW[l]) < 16 * u
        assert np.linalg.norm(gbb[l] - gb[l]) / np.linalg.norm(gb[l]) < 16 * u


def test_bf16_mode_exact_on_representable_first_layer():
    # with bf16-representable inputs and weights the rounding of the operands
    # changes nothing in the first pre-activation
    W, b = mlp.init(seed=7)
    W = [mlp.bf16(w) for w in W]
    x = mlp.bf16(np.random.default_rng(8).normal(size=(5, 6)))
    _, _, pre = mlp.forward(W, b, x, keep=True)
    _, _, preb = mlp.forward(W, b, x, keep=True, rnd=mlp.bf16)
    np.testing.assert_array_equal(pre[0], preb[0])
