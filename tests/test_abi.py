"""Host-side checks of the C ABI: the library loads, exports every entry
point include/cpm.h declares, and validates models without a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2312_09317_amd import cpm, inputs

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cpm.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*|void)\s*\**\s*(cpm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = cpm.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(cpm.EXPORTS)


def test_params_struct_layout_matches_header(tmp_path):
    # offsets of cpm_params as the C compiler lays them out from include/cpm.h
    fields = [f[0] for f in cpm.cpm_params._fields_]
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    lines.append('printf("%zu\\n", sizeof(cpm_params));')
    for f in fields:
        lines.append(f'printf("%zu\\n", offsetof(cpm_params, {f}));')
    lines.append('return 0; }')
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(cpm.cpm_params)
    for f, off in zip(fields, vals[1:]):
        assert getattr(cpm.cpm_params, f).offset == off, f


def _params(**kw):
    w = inputs.config1(L=32, grid=3, n_mcs=1)
    return cpm.Params.from_workload(w, **kw), w


def test_validate_accepts_workloads():
    p, w = _params()
    assert cpm.cpm_validate(p, w.n_cells) == cpm.CPM_OK
    w0 = inputs.config0()
    assert cpm.cpm_validate(cpm.Params.from_workload(w0), w0.n_cells) == cpm.CPM_OK
    nbytes = cpm.cpm_workspace_bytes(p, w.n_cells)
    assert nbytes > 8 * (w.n_cells + 1) * 2
    assert nbytes % 256 == 0


@pytest.mark.parametrize("change,code", [
    (dict(sub=3), cpm.CPM_EINVAL),             # 32 not divisible by 6
    (dict(attempts=3), cpm.CPM_EINVAL),        # 3 does not divide 8
    (dict(ndim=4), cpm.CPM_EINVAL),
    (dict(temperature=0.0), cpm.CPM_EINVAL),
    (dict(temperature=float("nan")), cpm.CPM_EINVAL),
    (dict(temperature=500.0), cpm.CPM_ENOTSUP),
    (dict(obstacle_type=7), cpm.CPM_EINVAL),
    (dict(J=[[0, 1e6], [1e6, 0]]), cpm.CPM_ERANGE),
    (dict(J=[[0, 1.0], [2.0, 0]]), cpm.CPM_EINVAL),  # asymmetric
    (dict(lambda_act=[0, 1.0], max_act=[0, 5], sub=1), cpm.CPM_EINVAL),
    (dict(lambda_act=[0, 1.0], max_act=[0, 300]), cpm.CPM_EINVAL),
    (dict(lambda_act=[0, 1.0], max_act=[3, 5]), cpm.CPM_EINVAL),
    (dict(lambda_persistence=[0, 40.0], persistence_mu=[0, 0.9], persistence_dt=0), cpm.CPM_EINVAL),
    (dict(lambda_persistence=[0, 40.0], persistence_mu=[0, 1.5], persistence_dt=5), cpm.CPM_EINVAL),
    (dict(lambda_persistence=[0, 40.0], persistence_mu=None, persistence_dt=5), cpm.CPM_EINVAL),
    (dict(lambda_persistence=[0, 1e6], persistence_mu=[0, 0.5], persistence_dt=5), cpm.CPM_ERANGE),
    (dict(lambda_persistence=[0, 40.0], persistence_mu=[0, 0.5], persistence_dt=5, dims=(2, 32, 32), sub=1),
     cpm.CPM_EINVAL),                          # an axis of 2 sites makes Moore offsets ambiguous
])
def test_validate_rejects(change, code):
    p, w = _params(**change)
    assert cpm.cpm_validate(p, w.n_cells) == code
    with pytest.raises(cpm.CpmError) as e:
        cpm.cpm_workspace_bytes(p, w.n_cells)
    assert e.value.code == code
    assert cpm.load().cpm_last_error()  # a message is set


def test_persistence_workspace_and_batches():
    p, w = _params()
    q, _ = _params(lambda_persistence=[0, 40.0], persistence_mu=[0, 0.95], persistence_dt=15)
    assert cpm.cpm_validate(q, w.n_cells) == cpm.CPM_OK
    # directions (int4) + 16 history centroids (3 x int64) + centroid sums per label
    extra = cpm.cpm_workspace_bytes(q, w.n_cells) - cpm.cpm_workspace_bytes(p, w.n_cells)
    labels = w.n_cells + 1
    assert extra >= labels * (16 + 16 * 24 + 3 * 8)
    with pytest.raises(cpm.CpmError) as e:
        cpm.cpm_batch_workspace_bytes([q], [w.n_cells])
    assert e.value.code == cpm.CPM_ENOTSUP
    wc = inputs.collective_3d(L=32, n_mcs=1)
    assert cpm.cpm_validate(cpm.Params.from_workload(wc), wc.n_cells) == cpm.CPM_OK
    # incremental centroid sums: also a reference point (int4) per label
    r, _ = _params(lambda_persistence=[0, 40.0], persistence_mu=[0, 0.95], persistence_dt=15,
                   persistence_centroids="incremental")
    assert cpm.cpm_validate(r, w.n_cells) == cpm.CPM_OK
    assert cpm.cpm_workspace_bytes(r, w.n_cells) - cpm.cpm_workspace_bytes(p, w.n_cells) >= extra
    bad, _ = _params(lambda_persistence=[0, 40.0], persistence_mu=[0, 0.95], persistence_dt=15,
                     persistence_centroids=2)
    assert cpm.cpm_validate(bad, w.n_cells) == cpm.CPM_EINVAL


class _FakeDevicePtr:
    # stands for a device tensor: only its address is read by validation
    def __init__(self, addr):
        self.addr = addr

    def data_ptr(self):
        return self.addr


def test_chemotaxis_validation():
    p, w = _params(lambda_chemotaxis=[0, 10.0])  # no field
    assert cpm.cpm_validate(p, w.n_cells) == cpm.CPM_EINVAL
    p, w = _params(lambda_chemotaxis=[0, 10.0], chemotaxis_field=_FakeDevicePtr(1 << 20))
    assert cpm.cpm_validate(p, w.n_cells) == cpm.CPM_OK
    p, w = _params(lambda_chemotaxis=[0, 10.0], chemotaxis_field=_FakeDevicePtr((1 << 20) + 2))
    assert cpm.cpm_validate(p, w.n_cells) == cpm.CPM_EINVAL  # not 4-byte aligned
    p, w = _params(lambda_chemotaxis=[0, 1e6], chemotaxis_field=_FakeDevicePtr(1 << 20))
    assert cpm.cpm_validate(p, w.n_cells) == cpm.CPM_ERANGE
    # the workload generator's field: 2 int16 per site, unit length within rounding
    wc = inputs.chemotaxis_2d()
    f = wc.C_field.reshape(-1, 2).astype(np.float64) / 16384
    assert f.shape[0] == wc.n_sites and np.abs(np.hypot(f[:, 0], f[:, 1]) - 1).max() < 1e-4


def test_validate_rejects_bad_cell_count_and_null():
    p, w = _params()
    assert cpm.cpm_validate(p, -1) == cpm.CPM_EINVAL
    assert cpm.load().cpm_validate(None, 5) == cpm.CPM_EINVAL


def test_init_rejects_small_workspace_without_touching_device():
    p, w = _params()
    lib = cpm.load()
    h = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(4096)  # never dereferenced: the size check fails first
    rc = lib.cpm_init(ctypes.byref(p.c), fake, fake, w.n_cells, None, fake, 16, None, ctypes.byref(h))
    assert rc == cpm.CPM_ENOMEM
    assert h.value is None


def test_strerror():
    lib = cpm.load()
    for c in range(6):
        assert lib.cpm_strerror(c)


EMU_HEADER = os.path.join(os.path.dirname(HEADER), "emu.h")


def test_emu_exports_every_declared_symbol():
    from paper_2312_09317_amd import emu
    text = open(EMU_HEADER).read()
    names = sorted(set(re.findall(r"^\s*int\s+(emu_\w+)\s*\(", text, re.M)))
    assert len(names) >= 10
    lib = emu.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(emu.EXPORTS)


def test_emu_host_calls_without_device():
    from paper_2312_09317_amd import emu
    # 6*256 + 256 + 2 * (256*256 + 256) + 8*256 + 8
    assert emu.emu_param_count() == 135432
    small, big = emu.emu_workspace_bytes(1), emu.emu_workspace_bytes(65536)
    assert small % 256 == 0 and big > 256 * 65536 * 2 * 6
    assert small < big
    for bad in (0, -1, (1 << 20) + 1):
        with pytest.raises(cpm.CpmError) as e:
            emu.emu_workspace_bytes(bad)
        assert e.value.code == cpm.CPM_EINVAL
    lib = emu.lib()
    h = ctypes.c_void_p(0)
    assert lib.emu_init(64, None, 1 << 20, None, ctypes.byref(h)) == cpm.CPM_EINVAL
    assert lib.emu_forward(None, None, 1, None, None) == cpm.CPM_EINVAL
    assert lib.emu_adam(None, None, 1e-3, None) == cpm.CPM_EINVAL


def test_emu_pack_round_trip():
    from paper_2312_09317_amd import emu
    from oracle import mlp
    W, b = mlp.init(seed=2)
    p = emu.pack(W, b)
    assert p.size == 135432 and p.dtype == np.float32
    W2, b2 = emu.unpack(p)
    for l in range(4):
        np.testing.assert_array_equal(W2[l], W[l].astype(np.float32))
        np.testing.assert_array_equal(b2[l], b[l].astype(np.float32))
