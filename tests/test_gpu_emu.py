"""GPU parity of the emulator kernels (bf16 matrix cores, fp32 accumulation)
against the FP64 reference in oracle/mlp.py, through the C ABI.

Tolerances (normwise relative, u = 2^-9 the bf16 unit roundoff):
* against the reference that rounds the same operands to bf16: 2e-3 for
  outputs and gradients (fp32 vs fp64 accumulation order, and the odd
  operand that rounds to the neighbouring bf16 value);
* against the exact FP64 reference: 8u for outputs (two rounded operands per
  product, four layers), 16u for gradients (one more rounded operand per
  layer on the way back).
Adam is elementwise fp32 arithmetic: 1e-5 relative.

Element by element, each output must also lie within 16u of the magnitude
bound m = |W4| g(|W3| g(|W2| g(|W1| |x| + |b1|) + |b2|) + |b3|) + |b4|
(g(v) = 1.13 v bounds the exact GELU's slope) of the exact FP64 output:
operands rounded to bf16 (relative u each) and fp32 sums, propagated through
four layers.  And no output row or column may stray from the bf16-rounded
reference by more than 2e-2 of that column's rms, so that one wrong row,
column or edge tile cannot hide inside a norm.
"""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

U = 2.0 ** -9


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _emu(torch, max_batch=4096):
    from paper_2312_09317_amd import emu
    e = emu.Emulator(max_batch)
    return emu, e


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _magnitude(W, b, x):
    """Per-element scale of the forward pass: |W| |.| chained with the GELU slope bound."""
    a = np.abs(x)
    for l in range(len(W)):
        a = np.abs(W[l]) @ a.T
        a = a.T + np.abs(b[l])
        if l < len(W) - 1:
            a = 1.13 * a
    return a


def _elementwise(y, ref_exact, ref_b, W, b, x):
    bound = 16 * U * _magnitude(W, b, x)
    bad = np.abs(y - ref_exact) > bound
    assert not bad.any(), f"{int(bad.sum())} outputs beyond the elementwise bound, first {np.argwhere(bad)[:3]}"
    scale = np.sqrt(np.mean(ref_b ** 2, axis=0)) + 1e-30
    err = np.abs(y - ref_b) / scale
    assert err.max(axis=0).max() < 2e-2, f"column errors {err.max(axis=0)}"
    assert err.max(axis=1).max() < 2e-2, f"worst row {int(np.argmax(err.max(axis=1)))}"


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 6))
    t = np.tanh(x @ rng.normal(size=(6, 8))) + 0.1 * rng.normal(size=(n, 8))
    return x, t


@pytest.mark.parametrize("n", [1, 63, 1000, 4096])
def test_forward_matches_oracle(torch, n):
    emu, e = _emu(torch)
    W, b = mlp.init(seed=11)
    for l in range(4):  # non-zero biases
        b[l] = np.random.default_rng(l).normal(scale=0.1, size=b[l].shape)
    e.set_params(emu.pack(W, b))
    x, _ = _data(n, 3)
    y = e.forward(x).cpu().numpy().astype(np.float64)
    # the GPU used the float32 parameters and inputs
    W32, b32 = emu.unpack(emu.pack(W, b))
    x32 = x.astype(np.float32).astype(np.float64)
    ref_b = mlp.forward(W32, b32, x32, rnd=mlp.bf16)
    ref = mlp.forward(W32, b32, x32)
    assert np.all(np.isfinite(y))
    assert _rel(y, ref_b) < 2e-3
    assert _rel(y, ref) < 8 * U
    _elementwise(y, ref, ref_b, W32, b32, x32)
    e.close()


def test_fit_norm_and_denormalised_forward(torch):
    emu, e = _emu(torch)
    W, b = mlp.init(seed=12)
    e.set_params(emu.pack(W, b))
    rng = np.random.default_rng(4)
    x = rng.normal(size=(500, 6)) * [1, 2, 3, 4, 5, 0.1] + [10, -3, 0, 2, 7, 0.5]
    t = rng.normal(size=(500, 8)) * np.arange(1, 9) + np.arange(8)
    x32, t32 = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    ref_norm = np.concatenate([x32.mean(0), x32.std(0), t32.mean(0), t32.std(0), np.zeros(8)])
    e.fit_norm(x, t)
    norm = e.norm().cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(norm, ref_norm, rtol=1e-6, atol=1e-6)
    # forward with a normalisation set from the host
    n32 = ref_norm.astype(np.float32).astype(np.float64)
    e.set_norm(n32)
    y = e.forward(x).cpu().numpy().astype(np.float64)
    W32, b32 = emu.unpack(emu.pack(W, b))
    xn = mlp.normalise(x32, n32[:6], n32[6:12])
    ref = mlp.denormalise(mlp.forward(W32, b32, xn, rnd=mlp.bf16), n32[12:20], n32[20:28])
    assert _rel(y - n32[12:20], ref - n32[12:20]) < 2e-3


@pytest.mark.parametrize("n", [1, 200, 1000, 2500])  # 2500: weight gradients split over K with a ragged last part
def test_gradients_match_oracle(torch, n):
    emu, e = _emu(torch)
    W, b = mlp.init(seed=13)
    for l in range(4):
        b[l] = np.random.default_rng(10 + l).normal(scale=0.1, size=b[l].shape)
    e.set_params(emu.pack(W, b))
    x, t = _data(n, 5)
    g, loss = e.grads(x, t)
    gW, gb = emu.unpack(g.cpu().numpy())
    W32, b32 = emu.unpack(emu.pack(W, b))
    x32, t32 = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    rW, rb = mlp.grads(W32, b32, x32, t32, rnd=mlp.bf16)
    eW, eb = mlp.grads(W32, b32, x32, t32)
    for l in range(4):
        assert _rel(gW[l], rW[l]) < 2e-3, ("W", l)
        assert _rel(gb[l], rb[l]) < 2e-3, ("b", l)
        assert _rel(gW[l], eW[l]) < 16 * U, ("W exact", l)
        assert _rel(gb[l], eb[l]) < 16 * U, ("b exact", l)
    ref_loss = mlp.loss(W32, b32, x32, t32, rnd=mlp.bf16)
    assert abs(float(loss.item()) - ref_loss) <= 2e-3 * ref_loss
    e.close()


def test_adam_matches_oracle(torch):
    emu, e = _emu(torch)
    W, b = mlp.init(seed=14)
    p0 = emu.pack(W, b)
    e.set_params(p0)
    rng = np.random.default_rng(7)
    opt = mlp.Adam(*emu.unpack(p0), lr=1e-3)
    params = [w.copy() for w in emu.unpack(p0)[0]] + [v.copy() for v in emu.unpack(p0)[1]]
    lrs = [1e-3, 1e-3, 5e-4]
    for step, lr in enumerate(lrs):
        g32 = (rng.normal(size=p0.size) * 10.0 ** rng.uniform(-6, 0, size=p0.size)).astype(np.float32)
        e.adam(lr, grad=torch.as_tensor(g32, device="cuda"))
        gW, gb = emu.unpack(g32)
        opt.lr = lr
        params = opt.step(params, gW + gb)
    assert e.steps == len(lrs)
    got = e.params().cpu().numpy().astype(np.float64)
    ref = emu.pack(params[:4], params[4:]).astype(np.float64)  # float32 of the FP64 result
    ref64 = np.concatenate([np.concatenate([w.reshape(-1), v]) for w, v in zip(params[:4], params[4:])])
    np.testing.assert_allclose(got, ref64, rtol=1e-5, atol=1e-8)
    assert np.max(np.abs(got - ref)) < 1e-5
    # the bf16 copies follow the master parameters: a forward pass after the
    # updates equals the reference forward pass with the updated parameters
    x, _ = _data(300, 8)
    y = e.forward(x).cpu().numpy().astype(np.float64)
    Wn, bn = emu.unpack(got.astype(np.float32))
    assert _rel(y, mlp.forward(Wn, bn, x.astype(np.float32).astype(np.float64), rnd=mlp.bf16)) < 2e-3
    e.close()


def test_train_step_is_grads_then_adam(torch):
    emu, e = _emu(torch)
    W, b = mlp.init(seed=15)
    p0 = emu.pack(W, b)
    x, t = _data(700, 9)
    e.set_params(p0)
    g, _ = e.grads(x, t)
    e.adam(2e-3, grad=g.clone())
    p_two = e.params().clone()
    e.set_params(p0)
    xd = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    td = torch.as_tensor(t, dtype=torch.float32, device="cuda")
    e.train_step(xd, td, 2e-3)
    torch.testing.assert_close(e.params(), p_two, rtol=0, atol=0)
    e.close()


def test_training_reduces_loss_like_oracle(torch):
    emu, e = _emu(torch)
    W, b = mlp.init(seed=16)
    x, t = _data(1024, 10)
    e.set_params(emu.pack(W, b))
    losses = e.fit(x, t, epochs=30, batch=256, lr=2e-3, seed=1)
    assert losses[-1] < 0.25 * losses[0]
    # oracle on the same mini-batch schedule for the first two epochs
    W32, b32 = emu.unpack(emu.pack(W, b))
    opt = mlp.Adam(W32, b32, lr=2e-3)
    params = list(W32) + list(b32)
    x32, t32 = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(1))
    ref_losses = []
    for _ in range(2):
        perm = rng.permutation(len(x))
        ls = []
        for s in range(0, len(x), 256):
            idx = perm[s:s + 256]
            ls.append(mlp.loss(params[:4], params[4:], x32[idx], t32[idx], rnd=mlp.bf16))
            gW, gb = mlp.grads(params[:4], params[4:], x32[idx], t32[idx], rnd=mlp.bf16)
            params = opt.step(params, gW + gb)
        ref_losses.append(np.mean(ls))
    np.testing.assert_allclose(losses[:2], ref_losses, rtol=2e-2)
    e.close()


def test_errors(torch):
    from paper_2312_09317_amd import cpm
    emu, e = _emu(torch, max_batch=100)
    x = torch.zeros((101, 6), dtype=torch.float32, device="cuda")
    y = torch.zeros((101, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(cpm.CpmError) as err:
        emu.emu_forward(e.handle, x, 101, y, e.stream)
    assert err.value.code == cpm.CPM_EINVAL
    with pytest.raises(cpm.CpmError):
        emu.emu_forward(e.handle, x, 0, y, e.stream)
    with pytest.raises(cpm.CpmError):
        emu.emu_adam(e.handle, None, 0.0, e.stream)
    with pytest.raises(cpm.CpmError):
        emu.emu_adam(e.handle, None, float("nan"), e.stream)
    # a valid call still works after the rejected ones
    e.forward(x[:100])
    torch.cuda.synchronize()
    e.close()


def test_log_targets(torch):
    # targets spanning decades, some zero: columns in the mask are learnt as
    # log(t + off), off = (geometric mean of the column's positive values) / 100
    emu, e = _emu(torch)
    W, b = mlp.init(seed=17)
    e.set_params(emu.pack(W, b))
    rng = np.random.default_rng(9)
    x = rng.normal(size=(700, 6))
    t = np.exp(rng.normal(size=(700, 8)) * 2.0) * np.arange(1, 9)
    t[::7, 3] = 0.0
    mask = 0b11111010
    e.fit_norm(x, t, log_mask=mask)
    norm = e.norm().cpu().numpy().astype(np.float64)
    x32, t32 = x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    geo = np.array([np.exp(np.log(c[c > 0]).mean()) for c in t32.T])
    off = np.where([(mask >> j) & 1 for j in range(8)], geo / 100.0, 0.0)
    u = np.where(off > 0, np.log(t32 + np.where(off > 0, off, 1.0)), t32)
    np.testing.assert_allclose(norm[:12], np.concatenate([x32.mean(0), x32.std(0)]), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(norm[28:], off, rtol=1e-6)
    np.testing.assert_allclose(norm[12:20], u.mean(0), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(norm[20:28], u.std(0), rtol=1e-5)
    # outputs come back through exp(.) - off
    n32 = np.concatenate([x32.mean(0), x32.std(0), u.mean(0), u.std(0), off]).astype(np.float32).astype(np.float64)
    e.set_norm(n32)
    y = e.forward(x).cpu().numpy().astype(np.float64)
    W32, b32 = emu.unpack(emu.pack(W, b))
    z = mlp.denormalise(mlp.forward(W32, b32, mlp.normalise(x32, n32[:6], n32[6:12]), rnd=mlp.bf16),
                        n32[12:20], n32[20:28])
    with np.errstate(over="ignore"):  # both branches are evaluated; the log columns are small
        ref = np.where(n32[28:] > 0, np.exp(z) - n32[28:], z)
    assert _rel(np.log(np.abs(y) + 1.0), np.log(np.abs(ref) + 1.0)) < 2e-3
    # the loss is taken on the transformed, z-scored targets
    _, loss = e.grads(x, t)
    tn = mlp.normalise(u, n32[12:20], n32[20:28])
    ref_loss = mlp.loss(W32, b32, mlp.normalise(x32, n32[:6], n32[6:12]), tn, rnd=mlp.bf16)
    assert abs(float(loss.item()) - ref_loss) <= 5e-3 * ref_loss
    e.close()
