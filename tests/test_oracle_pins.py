"""Pins of the CPU oracle against facts fixed outside it: an independent
library implementation of Philox, closed forms of exp and of box surfaces,
the full Hamiltonian of eq. 1 / eq. 3, and the invariants the paper states.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2312_09317_amd import inputs
from tests import hamiltonian as ham

HELPER_SRC = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_ref.cpp")
HELPER_LIB = os.path.join(os.path.dirname(__file__), "helpers", "_build", "librocrand_philox_ref.so")


def rocrand_ref():
    if not os.path.exists(HELPER_LIB) or os.path.getmtime(HELPER_LIB) < os.path.getmtime(HELPER_SRC):
        os.makedirs(os.path.dirname(HELPER_LIB), exist_ok=True)
        subprocess.run(["hipcc", "-O2", "-shared", "-fPIC", "--offload-arch=gfx950", HELPER_SRC,
                        "-o", HELPER_LIB], check=True)
    lib = ctypes.CDLL(HELPER_LIB)
    lib.ref_philox4x32_10.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_long]
    return lib


def rocrand_philox(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(ctr)
    rocrand_ref().ref_philox4x32_10(ctr.ctypes.data, key.ctypes.data, out.ctypes.data, len(ctr))
    return out


# ------------------------------------------------------------------ Philox

def test_philox_matches_rocrand():
    rng = np.random.default_rng(7)
    n = 2000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # structured counters like the sweep's: (area, mcs, activation<<8|j, lattice id)
    ctr[:100] = np.stack([np.arange(100), np.full(100, 3), np.full(100, 5 << 8), np.zeros(100)], 1)
    ctr[100] = [0, 0, 0, 0]
    key[100] = [0, 0]
    ctr[101] = [0xFFFFFFFF] * 4
    key[101] = [0xFFFFFFFF] * 2
    ref = rocrand_philox(ctr, key)
    ours = np.stack([oracle.philox(ctr[i], key[i]) for i in range(n)])
    np.testing.assert_array_equal(ours, ref)


def test_philox_uniform_chi2():
    key = np.array([1, 0], dtype=np.uint32)
    vals = np.stack([oracle.philox([a, 0, 0, 0], key) for a in range(20000)]).ravel()
    hist = np.bincount(vals >> 26, minlength=64)  # top 6 bits
    expected = vals.size / 64
    chi2 = float(np.sum((hist - expected) ** 2 / expected))
    assert chi2 < 120.0  # 63 dof; p ~ 3e-5


# ------------------------------------------------------------------ acceptance tables (eq. 2)

@pytest.mark.parametrize("T", [1.0, 3.0, 20.0, 80.0])
def test_threshold_tables_closed_form(T):
    TI, TM, TL = oracle.tables(T)
    h = np.arange(len(TI))
    # entries are floor(2^32 e^{-x}): compare to the closed form computed here
    assert np.all(np.abs(TI.astype(np.float64) - np.floor(np.exp(-h / T) * 2**32)) <= 1)
    assert TI[0] == 2**32 and TM[0] == 2**32 and TL[0] == 2**32
    # the table ends where 2^32 e^{-h/T} drops below 1
    assert np.exp(-len(TI) / T) * 2**32 < 1.0 + 1e-9
    assert np.exp(-(len(TI) - 1) / T) * 2**32 >= 1.0 - 1e-9
    assert np.all(np.diff(TI.astype(np.int64)) <= 0)


@pytest.mark.parametrize("T", [3.0, 20.0, 80.0])
def test_threshold_vs_exp(T):
    rng = np.random.default_rng(1)
    dh = np.concatenate([
        rng.integers(1, int(40 * T * 65536), size=20000),
        np.arange(1, 3000),
        np.arange(1, 60) * 65536,
        [int(22 * T * 65536), int(23 * T * 65536)],
    ]).astype(np.int64)
    thr = oracle.threshold(T, dh).astype(np.float64)
    exact = np.exp(-dh / (65536.0 * T)) * 2**32
    # three floors of values <= 2^32 lose at most 3 units of 2^-32
    assert np.all(thr <= exact + 1e-6 * np.maximum(exact, 1))
    assert np.all(exact - thr <= 3.0 + 1e-9 * exact)
    # whole-energy steps reproduce TI exactly
    TI, _, _ = oracle.tables(T)
    k = np.arange(len(TI))
    np.testing.assert_array_equal(oracle.threshold(T, k * 65536)[1:], TI[1:])
    # non-increasing in dH up to one unit: the floors of the composed tables
    # can make a step at a table boundary rise by one unit of 2^-32
    order = np.argsort(dh)
    assert np.all(np.diff(oracle.threshold(T, dh[order]).astype(np.int64)) <= 1)
    # non-positive changes always accepted
    assert np.all(oracle.threshold(T, np.array([0, -5, -2**40])) == 2**32)


# ------------------------------------------------------------------ counters (V, S)

@pytest.mark.parametrize("a,b", [(50, 50), (10, 10), (3, 7), (1, 1), (2, 9)])
def test_surface_closed_form_2d(a, b):
    # a box of a x b sites in 2D Moore-8: S = 9ab - (3a-2)(3b-2) = 6(a+b) - 4
    lat = np.zeros((1, 64, 64), dtype=np.int32)
    lat[0, 5:5 + b, 7:7 + a] = 1
    m = oracle.Model(2, (64, 64), np.zeros((2, 2)), [0, 0], [0, 0])
    V, S = oracle.recount(m, lat, 1)
    assert V[1] == a * b
    assert S[1] == 6 * (a + b) - 4
    if (a, b) == (50, 50):
        # the paper's 2D target A=600 for V=2500 sits just above a square's 596
        assert S[1] == 596


@pytest.mark.parametrize("a,b,c", [(5, 5, 6), (8, 8, 8), (1, 1, 1), (3, 4, 5)])
def test_surface_closed_form_3d(a, b, c):
    # a box in 3D Moore-26: S = 27abc - (3a-2)(3b-2)(3c-2)
    lat = np.zeros((20, 20, 20), dtype=np.int32)
    lat[2:2 + c, 3:3 + b, 4:4 + a] = 1
    m = oracle.Model(3, (20, 20, 20), np.zeros((2, 2)), [0, 0], [0, 0])
    V, S = oracle.recount(m, lat, 1)
    assert V[1] == a * b * c
    assert S[1] == 27 * a * b * c - (3 * a - 2) * (3 * b - 2) * (3 * c - 2)


def test_ball_surface_target():
    g = np.arange(-8, 9)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    lat = np.zeros((24, 24, 24), dtype=np.int32)
    lat[4:21, 4:21, 4:21] = ((X * X + Y * Y + Z * Z) <= 24).astype(np.int32)
    m = oracle.Model(3, (24, 24, 24), np.zeros((2, 2)), [0, 0], [0, 0])
    V, S = oracle.recount(m, lat, 1)
    assert V[1] == 485
    assert S[1] == inputs.S_TARGET_BALL_V500


def test_ball_surface_target_v1000():
    # r^2 <= 38 (1021 voxels) is the digitised ball nearest to V = 1000
    # (r^2 <= 37 has 949)
    g = np.arange(-8, 9)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    r2 = X * X + Y * Y + Z * Z
    assert (r2 <= 37).sum() == 949 and (r2 <= 38).sum() == 1021
    lat = np.zeros((24, 24, 24), dtype=np.int32)
    lat[4:21, 4:21, 4:21] = (r2 <= 38).astype(np.int32)
    m = oracle.Model(3, (24, 24, 24), np.zeros((2, 2)), [0, 0], [0, 0])
    V, S = oracle.recount(m, lat, 1)
    assert V[1] == 1021
    assert S[1] == inputs.S_TARGET_BALL_V1000


@pytest.mark.parametrize("ndim,dims", [(2, (12, 8, 1)), (3, (6, 4, 8))])
def test_recount_matches_definition(ndim, dims):
    lat = inputs.random_labels(dims, 5, seed=3, p_obstacle=0.1)
    m = oracle.Model(ndim, dims[:ndim], np.zeros((2, 2)), [0, 0], [0, 0])
    V, S = oracle.recount(m, lat, 4)
    Vt, St = ham.counts(lat, 4, ndim)
    np.testing.assert_array_equal(V[1:], Vt[1:])
    np.testing.assert_array_equal(S[1:], St[1:])


# ------------------------------------------------------------------ local dH == H(after) - H(before)

def _multi_type_model(ndim, dims, with_surface=True, T=7.0):
    # types: 0 medium, 1..3 cells, 4 obstacle
    J = np.array([[0, 3, 5, 2.5, 1.5],
                  [3, 7, 1.25, 4, -2],
                  [5, 1.25, 9, 6, 0.5],
                  [2.5, 4, 6, 11, 3],
                  [1.5, -2, 0.5, 3, 0]])
    lv = [0, 2.5, 1.0, 3.75, 0]
    vt = [0, 6, 9, 4, 0]
    ls = [0, 0.5, 0.25, 1.5, 0] if with_surface else None
    st = [0, 20, 30, 14, 0] if with_surface else None
    return oracle.Model(ndim, dims[:ndim], J, lv, vt, ls, st, T=T, obstacle_type=4), J, lv, vt, ls, st


@pytest.mark.parametrize("ndim,dims,seed", [(2, (8, 12, 1), 1), (2, (4, 4, 1), 2), (3, (6, 4, 4), 3),
                                            (3, (4, 4, 4), 4), (2, (2, 6, 1), 5)])
def test_delta_h_identity(ndim, dims, seed):
    rng = np.random.default_rng(seed)
    m, J, lv, vt, ls, st = _multi_type_model(ndim, dims)
    n_cells = 7
    cell_type = np.array([0, 1, 2, 3, 1, 2, 3, 1], dtype=np.int32)
    lat = inputs.random_labels(dims, n_cells + 1, seed=seed, p_obstacle=0.1)
    if seed % 2 == 0:
        lat = inputs.random_blobs(dims, n_cells, seed=seed, fill=0.7, p_obstacle=0.05)
    N = lat.size
    offs = ham.moore(ndim)
    checked = 0
    for _ in range(300):
        t = int(rng.integers(N))
        flat = lat.reshape(-1)
        if flat[t] < 0:
            continue
        z, y, x = np.unravel_index(t, lat.shape)
        if rng.random() < 0.5:
            o = offs[rng.integers(len(offs))]
            src = np.ravel_multi_index(((z + o[0]) % lat.shape[0], (y + o[1]) % lat.shape[1],
                                        (x + o[2]) % lat.shape[2]), lat.shape)
            nl = flat[src]
            if nl < 0 or nl == flat[t]:
                continue
        else:  # any other label, as in the symmetric proposal
            src = -1
            nl = int(rng.integers(n_cells + 1))
            if nl == flat[t]:
                continue
        V, S = ham.counts(lat, n_cells, ndim)
        dh = oracle.delta_h(m, lat, cell_type, V, S, t, src, nl)
        lat2 = lat.copy().reshape(-1)
        lat2[t] = nl
        lat2 = lat2.reshape(lat.shape)
        h0 = ham.full_h(lat, cell_type, n_cells, ndim, J, lv, vt, ls, st, obstacle_type=4)
        h1 = ham.full_h(lat2, cell_type, n_cells, ndim, J, lv, vt, ls, st, obstacle_type=4)
        assert dh == h1 - h0, (t, nl)
        checked += 1
    assert checked > 100


# ------------------------------------------------------------------ invariants of the sweep

@pytest.mark.parametrize("ndim,dims,s,k", [(2, (16, 24, 1), 2, 1), (2, (12, 8, 1), 1, 1),
                                           (3, (8, 8, 12), 2, 1), (2, (16, 16, 1), 2, 4),
                                           (3, (8, 8, 8), 2, 8), (2, (24, 24, 1), 3, 3)])
def test_sweep_counters_equal_recount(ndim, dims, s, k):
    # the paper's guarantee: tracked cell sizes equal the lattice counts
    m, *_ = _multi_type_model(ndim, dims, T=6.0)
    m.c.s, m.c.k = s, k
    cell_type = np.array([0, 1, 2, 3, 1, 2, 3, 1], dtype=np.int32)
    lat = inputs.random_blobs(dims, 7, seed=11, fill=0.6, p_obstacle=0.05)
    st = oracle.State(m, lat, cell_type)
    obst = st.lattice < 0
    for _ in range(4):
        st.sweep(2)
        V, S = oracle.recount(m, st.lattice, 7)
        np.testing.assert_array_equal(st.V[1:], V[1:])
        np.testing.assert_array_equal(st.S[1:], S[1:])
        assert np.all((st.lattice < 0) == obst)  # obstacles never change
        assert st.V[1:].sum() + np.sum(st.lattice == 0) + obst.sum() == lat.size
    assert st.stats[2] > 0  # something was accepted


def test_resume_is_bit_identical():
    w = inputs.config0()
    m = oracle.Model(2, w.dims[:2], w.J, w.lambda_V, w.V_target, w.lambda_S, w.S_target, T=w.T, seed=w.seed)
    a = oracle.State(m, w.lattice, w.cell_type)
    a.sweep(6)
    b = oracle.State(m, w.lattice, w.cell_type)
    b.sweep(2)
    b.sweep(4)
    np.testing.assert_array_equal(a.lattice, b.lattice)
    np.testing.assert_array_equal(a.V, b.V)
    np.testing.assert_array_equal(a.S, b.S)


def test_seed_and_lattice_id_change_the_stream():
    w = inputs.config0()
    res = []
    for seed, lid in [(1, 0), (2, 0), (1, 1)]:
        m = oracle.Model(2, w.dims[:2], w.J, w.lambda_V, w.V_target, T=w.T, seed=seed, lattice_id=lid)
        st = oracle.State(m, w.lattice, w.cell_type)
        st.sweep(3)
        res.append(st.lattice.copy())
    assert not np.array_equal(res[0], res[1])
    assert not np.array_equal(res[0], res[2])


def test_invalid_inputs_rejected():
    w = inputs.config0()
    m = oracle.Model(2, (100, 100), w.J, w.lambda_V, w.V_target, T=w.T, s=3)  # 100 % 6 != 0
    st = oracle.State.__new__(oracle.State)
    with pytest.raises(ValueError):
        oracle.State(m, w.lattice, w.cell_type).sweep(1)
    m2 = oracle.Model(2, (100, 100), w.J, w.lambda_V, w.V_target, T=w.T, s=2, k=3)  # 3 does not divide 4
    with pytest.raises(ValueError):
        oracle.State(m2, w.lattice, w.cell_type).sweep(1)
    bad = w.lattice.copy()
    bad[0, 0, 0] = 99  # label beyond the cell count
    m3 = oracle.Model(2, (100, 100), w.J, w.lambda_V, w.V_target, T=w.T)
    with pytest.raises(ValueError):
        st = oracle.State.__new__(oracle.State)
        oracle.State(m3, bad, w.cell_type)


def test_contacts_two_squares_closed_form():
    # two a x a squares of types 1 and 2 sharing a full edge in medium: each
    # side sees 3 sites across the edge per row but 2 at the two end rows
    from oracle import contacts
    for a in (3, 5, 8):
        lat = np.zeros((1, 20, 30), dtype=np.int32)
        lat[0, 4:4 + a, 5:5 + a] = 1
        lat[0, 4:4 + a, 5 + a:5 + 2 * a] = 2
        m = contacts.contact_matrix(lat, np.array([0, 1, 2]), 3, 2)
        assert m[1, 2] == m[2, 1] == 3 * a - 2
        assert m[1, 1] == m[2, 2] == 0  # one cell per type
        # row sums are the cells' surfaces (no obstacles here)
        mo = oracle.Model(2, (30, 20), np.zeros((3, 3)), [0, 0, 0], [0, 0, 0])
        V, S = oracle.recount(mo, lat[0], 2)
        assert m[1].sum() == S[1] and m[2].sum() == S[2]
        assert m[0].sum() == m[:, 0].sum()


@pytest.mark.parametrize("ndim,dims", [(2, (24, 18, 1)), (3, (8, 10, 6))])
def test_contacts_row_sums_equal_recounted_surfaces(ndim, dims):
    # on random multi-type states with obstacles: symmetric, and each type's
    # row sum equals the summed surfaces of its cells less obstacle contacts
    from oracle import contacts
    lat = inputs.random_blobs(dims, 9, seed=21, fill=0.7, p_obstacle=0.0)
    types = np.array([0] + [1 + (i % 3) for i in range(9)])
    m = contacts.contact_matrix(lat, types, 4, ndim)
    np.testing.assert_array_equal(m, m.T)
    mo = oracle.Model(ndim, dims[:ndim], np.zeros((4, 4)), [0] * 4, [0] * 4)
    V, S = oracle.recount(mo, lat if ndim == 3 else lat[0], 9)
    for t in (1, 2, 3):
        assert m[t].sum() == sum(S[c] for c in range(1, 10) if types[c] == t)
    # brute force over every site and neighbour on a tiny lattice
    small = inputs.random_labels((4, 5, 1) if ndim == 2 else (3, 4, 3), 4, seed=3, p_obstacle=0.2)
    ts = np.array([0, 1, 2, 1])
    bf = np.zeros((3, 3), dtype=np.int64)
    Lz, Ly, Lx = small.shape
    offs = [(dz, dy, dx) for dz in ((-1, 0, 1) if ndim == 3 else (0,)) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if (dz, dy, dx) != (0, 0, 0)]
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                c = small[z, y, x]
                for dz, dy, dx in offs:
                    u = small[(z + dz) % Lz, (y + dy) % Ly, (x + dx) % Lx]
                    if c != u and c >= 0 and u >= 0:
                        bf[ts[c] if c > 0 else 0, ts[u] if u > 0 else 0] += 1
    np.testing.assert_array_equal(contacts.contact_matrix(small, ts, 3, ndim), bf)
