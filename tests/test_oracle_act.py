"""Pins of the oracle's Act extension (Methods, eq. 7-8): geometric mean of
the activity over a site's own cell within its Moore neighbourhood, the sign
of the energy term, and the activity bookkeeping of the sweep."""
import numpy as np
import pytest

import oracle
from paper_2312_09317_amd import inputs


def _model(ndim, dims, lam_act=300.0, max_act=30, T=20.0):
    # types: 0 medium, 1 motile cell, 2 non-motile cell
    J = np.array([[0, 10, 10], [10, 20, 20], [10, 20, 20]], dtype=float)
    return oracle.Model(ndim, dims[:ndim], J, [0, 25, 25], [0, 50, 50], [0, 0.5, 0.5], [0, 200, 200],
                        lambda_act=[0, lam_act, 0], max_act=[0, max_act, 0], T=T)


def _neigh(ndim):
    r = range(-1, 2)
    if ndim == 2:
        return [(0, dy, dx) for dy in r for dx in r if dy or dx]
    return [(dz, dy, dx) for dz in r for dy in r for dx in r if dz or dy or dx]


@pytest.mark.parametrize("ndim,a", [(2, 1), (2, 7), (3, 30), (3, 255), (2, 200)])
def test_gm_uniform(ndim, a):
    dims = (8, 8, 8 if ndim == 3 else 1)
    lat = np.ones((dims[2], dims[1], dims[0]), dtype=np.int32)
    act = np.full(lat.shape, a, dtype=np.uint8)
    m = _model(ndim, dims)
    g = oracle.gm_act(m, lat, [0, 1], act, 3 + 8 * (3 + 8 * (dims[2] // 2)))
    assert abs(g - a * 65536) <= 2


def test_gm_matches_fp64_geometric_mean():
    rng = np.random.default_rng(3)
    dims = (6, 6, 6)
    m = _model(3, dims)
    errs = []
    for trial in range(300):
        lat = rng.integers(1, 3, size=(6, 6, 6)).astype(np.int32)  # cells 1 and 2, both motile type 1
        act = rng.integers(1, 256, size=(6, 6, 6)).astype(np.uint8)
        z, y, x = 3, 2, 4
        site = x + 6 * (y + 6 * z)
        cell = lat[z, y, x]
        vals = [int(act[z, y, x])]
        for dz, dy, dx in _neigh(3):
            if lat[(z + dz) % 6, (y + dy) % 6, (x + dx) % 6] == cell:
                vals.append(int(act[(z + dz) % 6, (y + dy) % 6, (x + dx) % 6]))
        exact = np.exp(np.mean(np.log(vals))) * 65536
        g = oracle.gm_act(m, lat, [0, 1, 1], act, site)
        errs.append(abs(g - exact) / exact)
    assert max(errs) < 2.0 ** -14


def test_gm_zero_cases_and_own_cell_only():
    dims = (8, 8, 1)
    m = _model(2, dims)
    lat = np.zeros((1, 8, 8), dtype=np.int32)
    lat[0, 2:6, 2:6] = 1
    lat[0, 2:6, 6] = 2
    act = np.full(lat.shape, 9, dtype=np.uint8)
    ct = [0, 1, 2]  # cell 2 is non-motile
    assert oracle.gm_act(m, lat, ct, act, 0) == 0                    # medium
    assert oracle.gm_act(m, lat, ct, act, 6 + 8 * 3) == 0            # non-motile cell
    base = oracle.gm_act(m, lat, ct, act, 5 + 8 * 3)
    act2 = act.copy()
    act2[0, 3, 6] = 1                                                 # other cell's neighbour
    act2[0, 3, 1] = 200                                               # medium, not a neighbour
    assert oracle.gm_act(m, lat, ct, act2, 5 + 8 * 3) == base
    act3 = act.copy()
    act3[0, 4, 4] = 0                                                 # a zero in the own-cell set
    assert oracle.gm_act(m, lat, ct, act3, 5 + 8 * 3) == 0


def test_act_term_sign():
    # a copy from a high-activity source into a resting neighbour is favoured,
    # the opposite copy is penalised, and equal activities cancel
    dims = (12, 12, 1)
    m_act = _model(2, dims)
    m_off = _model(2, dims, lam_act=0.0)
    lat = np.zeros((1, 12, 12), dtype=np.int32)
    lat[0, 3:9, 2:6] = 1
    lat[0, 3:9, 6:10] = 2
    ct = [0, 1, 1]
    V = np.array([0, 24, 24])
    S = np.array([0, 100, 100])
    t = 6 + 12 * 5   # in cell 2, at the interface
    src = 5 + 12 * 5  # in cell 1
    for hi_src in (True, False):
        act = np.zeros(lat.shape, dtype=np.uint8)
        act[lat == 1] = 30 if hi_src else 2
        act[lat == 2] = 2 if hi_src else 30
        d1 = oracle.delta_h(m_act, lat, ct, V, S, t, src, 1, act)
        d0 = oracle.delta_h(m_off, lat, ct, V, S, t, src, 1, act)
        assert (d1 - d0 < 0) == hi_src
    act = np.full(lat.shape, 11, dtype=np.uint8)
    act[lat == 0] = 0
    d1 = oracle.delta_h(m_act, lat, ct, V, S, t, src, 1, act)
    d0 = oracle.delta_h(m_off, lat, ct, V, S, t, src, 1, act)
    assert abs(d1 - d0) <= 1
    # protrusion into medium: the target term vanishes, only -R * GM(source)
    t_med = 1 + 12 * 5
    src_c = 2 + 12 * 5
    act = np.full(lat.shape, 30, dtype=np.uint8)
    d1 = oracle.delta_h(m_act, lat, ct, V, S, t_med, src_c, 1, act)
    d0 = oracle.delta_h(m_off, lat, ct, V, S, t_med, src_c, 1, act)
    gm = oracle.gm_act(m_act, lat, ct, act, src_c)
    assert d1 - d0 == -((10 * 65536 * gm) >> 16)  # R = lambda_act / max_act = 10


@pytest.mark.parametrize("ndim,dims", [(2, (24, 24, 1)), (3, (12, 12, 8))])
def test_sweep_act_bookkeeping(ndim, dims):
    m = _model(ndim, dims, T=30.0)
    lat = inputs.random_blobs(dims, 6, seed=4, fill=0.6)
    ct = np.array([0, 1, 2, 1, 2, 1, 1], dtype=np.int32)
    st = oracle.State(m, lat, ct)
    st.sweep(1)
    a = st.act.reshape(-1)
    l0 = lat.reshape(-1)
    l1 = st.lattice
    assert set(np.unique(a)) <= {0, 29}
    motile = (l1 > 0) & (ct[np.maximum(l1, 0)] == 1)
    assert np.all(a[~motile] == 0)
    assert np.all(a[(l1 != l0) & motile] == 29)
    V, S = oracle.recount(m, st.lattice, 6)
    np.testing.assert_array_equal(st.V[1:], V[1:])
    np.testing.assert_array_equal(st.S[1:], S[1:])
    for _ in range(3):
        st.sweep(1)
    assert st.act.max() <= 29
    assert np.all(st.act[st.lattice <= 0] == 0)


def test_act_requires_sub_area_two():
    m = _model(2, (12, 12, 1))
    m.c.s = 1
    lat = inputs.random_blobs((12, 12, 1), 3, seed=4)
    with pytest.raises(ValueError):
        oracle.State(m, lat, [0, 1, 1, 1]).sweep(1)
