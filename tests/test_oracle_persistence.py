"""Pins of the oracle's persistence extension (Methods, eq. 5-6): direction
updates of cells moved by hand against closed forms, and the energy term's
sign and size for copies along, against and across a cell's direction."""
import math

import numpy as np
import pytest

import oracle


def _model(ndim, dims, mu=0.0, lam=40.0, dt=1):
    n = 2
    return oracle.Model(ndim, dims, np.zeros((n, n)), [0, 0], [0, 0], T=20.0,
                        lambda_P=[0.0, lam], mu_P=[0.0, mu], dt_P=dt)


def _square(L, x0, y0, a=4):
    lat = np.zeros((L, L), dtype=np.int32)
    for y in range(y0, y0 + a):
        for x in range(x0, x0 + a):
            lat[y % L, x % L] = 1
    return lat


TYPES = np.array([0, 1], dtype=np.int32)


def test_one_site_step_gives_unit_direction():
    m = _model(2, (32, 32))
    p = oracle.Persistence(m, _square(32, 5, 7), 1)
    P = p.update(_square(32, 6, 7), TYPES)
    assert tuple(P[1]) == (16384, 0, 0)
    P = p.update(_square(32, 6, 6), TYPES)  # now one step towards -y
    assert tuple(P[1]) == (0, -16384, 0)


def test_diagonal_step_and_periodic_wrap():
    m = _model(2, (32, 32))
    p = oracle.Persistence(m, _square(32, 30, 30), 1)  # straddles both boundaries
    P = p.update(_square(32, 31, 31), TYPES)
    r = round(16384 / math.sqrt(2))
    assert P[1, 0] == P[1, 1] and abs(P[1, 0] - r) <= 1 and P[1, 2] == 0


def test_mixing_weight_extremes():
    # mu = 1 keeps the previous direction (initially none); mu = 0.5 halves
    # the turn from +x towards +y (equal weights: the bisector)
    m = _model(2, (32, 32), mu=1.0)
    p = oracle.Persistence(m, _square(32, 5, 7), 1)
    assert tuple(p.update(_square(32, 6, 7), TYPES)[1]) == (0, 0, 0)
    m = _model(2, (32, 32), mu=0.5)
    p = oracle.Persistence(m, _square(32, 5, 7), 1)
    p.update(_square(32, 6, 7), TYPES)
    P = p.update(_square(32, 6, 8), TYPES)
    assert P[1, 0] == P[1, 1] and abs(P[1, 0] - round(16384 / math.sqrt(2))) <= 1


def test_lookback_over_dt_updates():
    # dt = 3: the displacement is taken over the last three updates (fewer
    # at the start, against the initial centroid); moving +1 in x each time
    # and -1 in y at the third step, the direction at update 4 is (3, -1)/|.|
    m = _model(2, (40, 40), dt=3)
    p = oracle.Persistence(m, _square(40, 5, 10), 1)
    steps = [(6, 10), (7, 10), (8, 9), (9, 9)]
    for x, y in steps:
        P = p.update(_square(40, x, y), TYPES)
    # update 4 looks back to update 1 (x=6, y=10): displacement (3, -1)
    d = np.array([3.0, -1.0]) / math.sqrt(10.0)
    np.testing.assert_allclose(P[1, :2] / 16384.0, d, atol=2e-4)


def test_dead_cell_has_no_direction():
    m = _model(2, (32, 32))
    p = oracle.Persistence(m, _square(32, 5, 7), 1)
    P = p.update(np.zeros((32, 32), dtype=np.int32), TYPES)
    assert tuple(P[1]) == (0, 0, 0)


@pytest.mark.parametrize("ndim", [2, 3])
def test_energy_term_along_against_across(ndim):
    # a cell with direction +x copying into the site in front of it, behind
    # it and beside it: -lambda, +lambda and 0 (lambda = 40 in 2^-16 units)
    dims = (16, 16, 16) if ndim == 3 else (16, 16)
    m = _model(ndim, dims, lam=40.0)
    shape = dims[::-1]
    lat = np.zeros(shape, dtype=np.int32)
    sl = tuple(slice(6, 10) for _ in range(ndim))
    lat[sl] = 1
    flat = lat.reshape(-1)
    V = np.array([0, flat.sum()], dtype=np.int64)
    S = np.array([0, 0], dtype=np.int64)
    P = np.zeros(6, dtype=np.int32)
    P[3] = 16384  # cell 1 points along +x
    Lx = dims[0]
    def site(x, y, z=0):
        return x + Lx * (y + dims[1] * z)
    z = 7 if ndim == 3 else 0
    lam = 40 * 65536
    cases = [(site(10, 7, z), site(9, 7, z), -lam),   # source inside, target ahead (+x)
             (site(5, 7, z), site(6, 7, z), +lam),    # target behind (-x)
             (site(7, 10, z), site(7, 9, z), 0)]      # target beside (+y)
    for t, src, want in cases:
        base = oracle.delta_h(m, flat, TYPES, V, S, t, src, 1)
        with_p = oracle.delta_h(m, flat, TYPES, V, S, t, src, 1, P=P)
        assert with_p - base == want, (t, src)
