"""ctypes binding of the emulator calls in libcpm (include/emu.h).

Argument marshalling only: every arithmetic step runs in the library's HIP
kernels.  Device buffers are torch tensors; calls enqueue on torch's current
stream of the tensors' device.
"""
import ctypes

import numpy as np

from . import cpm

EXPORTS = ("emu_param_count", "emu_workspace_bytes", "emu_init", "emu_set_params", "emu_get_params",
           "emu_set_norm", "emu_get_norm", "emu_fit_norm", "emu_forward", "emu_grads", "emu_adam",
           "emu_train_step", "emu_step_count", "emu_destroy")

N_IN, N_OUT, N_NORM = 6, 8, 36
SIZES = (6, 256, 256, 256, 8)

_bound = False


def lib():
    """libcpm with the emu_* signatures set."""
    global _bound
    l = cpm.load()
    if _bound:
        return l
    P, I32, F32, SZ, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t, ctypes.c_int64
    l.emu_param_count.argtypes = [ctypes.POINTER(I64)]
    l.emu_workspace_bytes.argtypes = [I32, ctypes.POINTER(SZ)]
    l.emu_init.argtypes = [I32, P, SZ, P, ctypes.POINTER(P)]
    l.emu_set_params.argtypes = [P, P, P]
    l.emu_get_params.argtypes = [P, P, P]
    l.emu_set_norm.argtypes = [P, P, P]
    l.emu_get_norm.argtypes = [P, P, P]
    l.emu_fit_norm.argtypes = [P, P, P, I32, I32, P]
    l.emu_forward.argtypes = [P, P, I32, P, P]
    l.emu_grads.argtypes = [P, P, P, I32, P, P, P]
    l.emu_adam.argtypes = [P, P, F32, P]
    l.emu_train_step.argtypes = [P, P, P, I32, F32, P, P]
    l.emu_step_count.argtypes = [P, ctypes.POINTER(I64)]
    l.emu_destroy.argtypes = [P]
    for f in EXPORTS:
        getattr(l, f).restype = ctypes.c_int
    _bound = True
    return l


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check(rc, where):
    if rc != cpm.CPM_OK:
        raise cpm.CpmError(rc, where)


# ---------------------------------------------------------------- C ABI, same names

def emu_param_count() -> int:
    v = ctypes.c_int64(0)
    _check(lib().emu_param_count(ctypes.byref(v)), "emu_param_count")
    return v.value


def emu_workspace_bytes(max_batch: int) -> int:
    v = ctypes.c_size_t(0)
    _check(lib().emu_workspace_bytes(max_batch, ctypes.byref(v)), "emu_workspace_bytes")
    return v.value


def emu_init(max_batch: int, d_workspace, workspace_bytes: int, stream: int) -> int:
    h = ctypes.c_void_p(0)
    _check(lib().emu_init(max_batch, _ptr(d_workspace), workspace_bytes, stream, ctypes.byref(h)), "emu_init")
    return h.value


def emu_set_params(h, d_params, stream):
    _check(lib().emu_set_params(h, _ptr(d_params), stream), "emu_set_params")


def emu_get_params(h, d_params, stream):
    _check(lib().emu_get_params(h, _ptr(d_params), stream), "emu_get_params")


def emu_set_norm(h, d_norm, stream):
    _check(lib().emu_set_norm(h, _ptr(d_norm), stream), "emu_set_norm")


def emu_get_norm(h, d_norm, stream):
    _check(lib().emu_get_norm(h, _ptr(d_norm), stream), "emu_get_norm")


def emu_fit_norm(h, d_x, d_t, n, log_mask, stream):
    _check(lib().emu_fit_norm(h, _ptr(d_x), _ptr(d_t), n, log_mask, stream), "emu_fit_norm")


def emu_forward(h, d_x, n, d_y, stream):
    _check(lib().emu_forward(h, _ptr(d_x), n, _ptr(d_y), stream), "emu_forward")


def emu_grads(h, d_x, d_t, n, d_grad, d_loss, stream):
    _check(lib().emu_grads(h, _ptr(d_x), _ptr(d_t), n, _ptr(d_grad), _ptr(d_loss), stream), "emu_grads")


def emu_adam(h, d_grad, lr, stream):
    _check(lib().emu_adam(h, _ptr(d_grad), lr, stream), "emu_adam")


def emu_train_step(h, d_x, d_t, n, lr, d_loss, stream):
    _check(lib().emu_train_step(h, _ptr(d_x), _ptr(d_t), n, lr, _ptr(d_loss), stream), "emu_train_step")


def emu_step_count(h) -> int:
    v = ctypes.c_int64(0)
    _check(lib().emu_step_count(h, ctypes.byref(v)), "emu_step_count")
    return v.value


def emu_destroy(h):
    lib().emu_destroy(h)


# ---------------------------------------------------------------- packing

def pack(W, b) -> np.ndarray:
    """Per-layer W (out x in) and b (out,) -> the packed float32 vector."""
    parts = []
    for w, v in zip(W, b):
        parts += [np.asarray(w, dtype=np.float32).reshape(-1), np.asarray(v, dtype=np.float32).reshape(-1)]
    return np.concatenate(parts)


def unpack(p):
    """Packed vector -> per-layer W and b (views into a float64 copy)."""
    p = np.asarray(p, dtype=np.float64)
    W, b, o = [], [], 0
    for i in range(len(SIZES) - 1):
        n_in, n_out = SIZES[i], SIZES[i + 1]
        W.append(p[o:o + n_in * n_out].reshape(n_out, n_in))
        o += n_in * n_out
        b.append(p[o:o + n_out])
        o += n_out
    return W, b


def norm_vector(x_mean, x_std, t_mean, t_std, t_off=None) -> np.ndarray:
    t_off = np.zeros(N_OUT) if t_off is None else t_off
    return np.concatenate([x_mean, x_std, t_mean, t_std, t_off]).astype(np.float32)


# ---------------------------------------------------------------- convenience wrapper

class Emulator:
    """An emulator handle with its workspace on `device`."""

    def __init__(self, max_batch: int, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.max_batch = int(max_batch)
        nbytes = emu_workspace_bytes(self.max_batch)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = emu_init(self.max_batch, self.workspace, nbytes, self.stream)
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    @property
    def stream(self) -> int:
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _dev(self, a, cols=None):
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
        if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
            raise ValueError(f"expected an (n, {cols}) array")
        return t

    def set_params(self, packed) -> None:
        emu_set_params(self.handle, self._dev(packed), self.stream)

    def params(self):
        out = self.torch.empty(emu_param_count(), dtype=self.torch.float32, device=self.device)
        emu_get_params(self.handle, out, self.stream)
        return out

    def set_norm(self, norm) -> None:
        emu_set_norm(self.handle, self._dev(norm), self.stream)

    def norm(self):
        out = self.torch.empty(N_NORM, dtype=self.torch.float32, device=self.device)
        emu_get_norm(self.handle, out, self.stream)
        return out

    def fit_norm(self, x, t, log_mask: int = 0) -> None:
        x, t = self._dev(x, N_IN), self._dev(t, N_OUT)
        emu_fit_norm(self.handle, x, t, x.shape[0], log_mask, self.stream)

    def forward(self, x):
        x = self._dev(x, N_IN)
        y = self.torch.empty((x.shape[0], N_OUT), dtype=self.torch.float32, device=self.device)
        emu_forward(self.handle, x, x.shape[0], y, self.stream)
        return y

    def grads(self, x, t):
        """(packed gradient, loss) of the mean squared error on one batch."""
        x, t = self._dev(x, N_IN), self._dev(t, N_OUT)
        g = self.torch.empty(emu_param_count(), dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        emu_grads(self.handle, x, t, x.shape[0], g, loss, self.stream)
        return g, loss

    def adam(self, lr: float, grad=None) -> None:
        emu_adam(self.handle, None if grad is None else self._dev(grad), lr, self.stream)

    def train_step(self, x, t, lr: float):
        """One Adam step on a batch; returns the loss before the step (device tensor)."""
        emu_train_step(self.handle, x, t, x.shape[0], lr, self._loss, self.stream)
        return self._loss

    def fit(self, x, t, epochs: int, batch: int, lr: float, seed: int = 0, lr_final=None):
        """Mini-batch Adam over (x, t) resident on the device, reshuffled each
        epoch from a seeded PCG64 stream; the learning rate decays
        geometrically from lr to lr_final (default lr) over the run.
        Returns the mean loss of each epoch."""
        torch = self.torch
        x, t = self._dev(x, N_IN), self._dev(t, N_OUT)
        n = x.shape[0]
        batch = min(batch, self.max_batch, n)
        rng = np.random.Generator(np.random.PCG64(seed))
        steps = epochs * ((n + batch - 1) // batch)
        decay = 1.0 if lr_final is None else (lr_final / lr) ** (1.0 / max(steps - 1, 1))
        losses, step = [], 0
        acc = torch.zeros(1, dtype=torch.float64, device=self.device)
        for _ in range(epochs):
            perm = torch.as_tensor(rng.permutation(n), device=self.device)
            xs, ts = x[perm].contiguous(), t[perm].contiguous()
            acc.zero_()
            nb = 0
            for s in range(0, n, batch):
                e = min(n, s + batch)
                loss = self.train_step(xs[s:e], ts[s:e], lr * decay ** step)
                acc += loss.double()
                nb += 1
                step += 1
            losses.append(float(acc.item()) / nb)
        return losses

    @property
    def steps(self) -> int:
        return emu_step_count(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            emu_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
