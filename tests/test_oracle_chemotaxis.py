"""Pins of the oracle's chemotaxis extension (Methods, eq. 4): the energy
term for copies along, against, across and diagonal to a fixed field, the
field read at the source (not the target), no term for medium copies, and a
single cell drifting along a uniform field in the serial CPM."""
import numpy as np
import pytest

import oracle

LAM = 10.0  # the paper's chemotaxis strength (its 2D chemotaxis settings)
TYPES = np.array([0, 1], dtype=np.int32)


def _model(ndim, dims, field, lam=LAM, **kw):
    n = 2
    return oracle.Model(ndim, dims, np.zeros((n, n)), [0, 0], [0, 0], T=kw.pop("T", 10.0),
                        lambda_C=[0.0, lam], C_field=field, **kw)


def _uniform(dims, vec):
    n = int(np.prod(dims))
    return np.tile(np.asarray(vec, dtype=np.int16), n)


def _dh(m, lat, t, src, new_label):
    V = np.zeros(2, dtype=np.int64)
    S = np.zeros(2, dtype=np.int64)
    return oracle.delta_h(m, lat.reshape(-1), TYPES, V, S, t, src, new_label)


def _site(dims, x, y, z=0):
    return x + dims[0] * (y + dims[1] * z)


@pytest.mark.parametrize("ndim", [2, 3])
def test_along_against_across(ndim):
    dims = (16, 16, 16) if ndim == 3 else (16, 16)
    full = dims if ndim == 3 else dims + (1,)
    one = [16384] + [0] * (ndim - 1)  # unit +x in 2^-14
    m = _model(ndim, dims, _uniform(dims, one))
    m0 = _model(ndim, dims, _uniform(dims, [0] * ndim))
    lat = np.zeros(full[::-1], dtype=np.int32)
    z = 8 if ndim == 3 else 0
    lat[z, 6:10, 6:10] = 1  # a 4 x 4 (x 1) cell, medium around it
    lam_q = round(LAM * 65536)
    src = _site(full, 9, 7, z)
    # +x: the cell extends along the field
    d = _dh(m, lat, _site(full, 10, 7, z), src, 1) - _dh(m0, lat, _site(full, 10, 7, z), src, 1)
    assert d == -lam_q
    # -x: a copy from the cell's left edge outwards, against the field
    src_l = _site(full, 6, 7, z)
    d = _dh(m, lat, _site(full, 5, 7, z), src_l, 1) - _dh(m0, lat, _site(full, 5, 7, z), src_l, 1)
    assert d == lam_q
    # +y: across the field
    src_t = _site(full, 7, 9, z)
    d = _dh(m, lat, _site(full, 7, 10, z), src_t, 1) - _dh(m0, lat, _site(full, 7, 10, z), src_t, 1)
    assert d == 0
    # +x+y: cos 45 degrees, the unit offset rounded to 2^-14 (11585)
    src_c = _site(full, 9, 9, z)
    d = _dh(m, lat, _site(full, 10, 10, z), src_c, 1) - _dh(m0, lat, _site(full, 10, 10, z), src_c, 1)
    assert d == -((lam_q * 11585 * 16384) >> 28)
    assert abs(d / lam_q + 2 ** -0.5) < 1e-4


def test_field_is_read_at_the_source():
    dims = (16, 16)
    field = np.zeros((16, 16, 2), dtype=np.int16)
    field[..., 1] = 16384           # +y everywhere ...
    field[7, 9] = (16384, 0)        # ... but +x at the source
    m = _model(2, dims, field.reshape(-1))
    m0 = _model(2, dims, np.zeros(16 * 16 * 2, dtype=np.int16))
    lat = np.zeros((1, 16, 16), dtype=np.int32)
    lat[0, 6:10, 6:10] = 1
    t, src = _site((16, 16, 1), 10, 7), _site((16, 16, 1), 9, 7)
    assert _dh(m, lat, t, src, 1) - _dh(m0, lat, t, src, 1) == -round(LAM * 65536)
    # a field at the target only changes nothing
    field2 = np.zeros((16, 16, 2), dtype=np.int16)
    field2[7, 10] = (16384, 0)
    m2 = _model(2, dims, field2.reshape(-1))
    assert _dh(m2, lat, t, src, 1) == _dh(m0, lat, t, src, 1)


def test_medium_copies_have_no_term():
    dims = (16, 16)
    m = _model(2, dims, _uniform(dims, [16384, 0]))
    m0 = _model(2, dims, _uniform(dims, [0, 0]))
    lat = np.zeros((1, 16, 16), dtype=np.int32)
    lat[0, 6:10, 6:10] = 1
    # medium at (5, 7) copies into the cell's edge site (6, 7): a retraction
    t, src = _site((16, 16, 1), 6, 7), _site((16, 16, 1), 5, 7)
    assert _dh(m, lat, t, src, 0) == _dh(m0, lat, t, src, 0)


def _centroid_x(lat, L):
    # minimum-image mean x of label 1 around its first site
    ys, xs = np.nonzero(lat[0] == 1)
    r = xs[0]
    d = (xs - r + L // 2) % L - L // 2
    return r + d.mean()


@pytest.mark.parametrize("sign", [1, -1])
def test_cell_drifts_along_a_uniform_field(sign):
    # serial CPM, one cell (V_target 100) in a uniform field along +-x: its
    # centroid moves the field's way, several sites over 60 MCS
    L = 48
    field = _uniform((L, L), [sign * 16384, 0])
    m = oracle.Model(2, (L, L), [[0, 10], [10, 20]], [0, 20], [0, 100], [0, 0.5], [0, 116], T=10.0,
                     seed=3, lambda_C=[0.0, 40.0], C_field=field)
    lat = np.zeros((1, L, L), dtype=np.int32)
    lat[0, 19:29, 19:29] = 1
    st = oracle.State(m, lat, TYPES)
    x0, moved = _centroid_x(st.lattice.reshape(1, L, L), L), 0.0
    for _ in range(60):
        st.serial_sweep(1)
        x1 = _centroid_x(st.lattice.reshape(1, L, L), L)
        moved += (x1 - x0 + L / 2) % L - L / 2
        x0 = x1
    assert sign * moved > 3.0, moved
