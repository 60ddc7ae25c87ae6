"""FP64 reference of the summary-statistics emulator (test infrastructure only).

A multilayer perceptron 6 -> 256 -> 256 -> 256 -> 8 with the exact (erf) GELU
after every hidden layer, trained on mean squared error with Adam.  Inputs and
outputs are z-scored with stored means and standard deviations.  Plain numpy
in float64: forward, backward by the chain rule, and the Adam update
(Kingma & Ba, 2015) with bias correction.

Weight layout: W[l] has shape (out, in), b[l] shape (out,); a layer computes
z = x @ W.T + b.

Precision: by default every step is float64.  With rnd=bf16 the forward and
backward passes round the operands of every matrix product to bfloat16
(weights, layer inputs and the gradients with respect to pre-activations)
where a bf16-operand, fp32-accumulating implementation rounds them; sums and
everything else stay float64.  This is the stated precision of the
emulator's matrix products, taken step by step.
"""
import math

import numpy as np

SIZES = (6, 256, 256, 256, 8)
_SQRT2 = math.sqrt(2.0)
_ERF = np.vectorize(math.erf)


def bf16(x):
    """Round to the nearest bfloat16 value (ties to even), via float32:
    keep the upper 16 bits of the float32 pattern after adding 0x7FFF plus
    the lowest kept bit.  Non-finite values pass through."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = np.isfinite(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = np.where(finite, r, u).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def _same(x):
    return x


def gelu(z):
    return 0.5 * z * (1.0 + _ERF(z / _SQRT2))


def gelu_grad(z):
    # d/dz [z Phi(z)] = Phi(z) + z phi(z)
    return 0.5 * (1.0 + _ERF(z / _SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init(seed=0, sizes=SIZES):
    """He-style uniform initialisation from a seeded PCG64 stream (the shared
    seeded input generator)."""
    from paper_2312_09317_amd.inputs import mlp_weights
    return mlp_weights(seed, sizes)


def forward(W, b, x, keep=False, rnd=_same):
    """x: (n, 6) already normalised.  Returns y (n, 8) and, if keep, the
    per-layer (rounded) inputs and pre-activations for the backward pass."""
    a = rnd(np.asarray(x, dtype=np.float64))
    acts, pre = [a], []
    for l in range(len(W)):
        z = a @ rnd(W[l]).T + b[l]
        pre.append(z)
        a = rnd(gelu(z)) if l < len(W) - 1 else z
        acts.append(a)
    return (a, acts, pre) if keep else a


def loss(W, b, x, t, rnd=_same):
    y = forward(W, b, x, rnd=rnd)
    return float(np.mean((y - t) ** 2))


def grads(W, b, x, t, rnd=_same):
    """Gradients of the mean squared error over all n x 8 outputs, by the
    chain rule from the output layer down."""
    y, acts, pre = forward(W, b, x, keep=True, rnd=rnd)
    n_out = y.size
    g = 2.0 * (y - t) / n_out  # dL/dy
    gW = [None] * len(W)
    gb = [None] * len(W)
    for l in range(len(W) - 1, -1, -1):
        dz = rnd(g if l == len(W) - 1 else g * gelu_grad(pre[l]))
        gW[l] = dz.T @ acts[l]
        gb[l] = dz.sum(axis=0)
        g = dz @ rnd(W[l])
    return gW, gb


class Adam:
    def __init__(self, W, b, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = [np.zeros_like(p) for p in W + b]
        self.v = [np.zeros_like(p) for p in W + b]

    def step(self, params, grads_):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (p, g) in enumerate(zip(params, grads_)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            out.append(p - self.lr * (self.m[i] / c1) / (np.sqrt(self.v[i] / c2) + self.eps))
        return out


def normalise(v, mean, std):
    return (np.asarray(v, dtype=np.float64) - mean) / std


def denormalise(v, mean, std):
    return np.asarray(v, dtype=np.float64) * std + mean
