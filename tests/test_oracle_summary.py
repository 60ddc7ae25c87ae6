"""Pins of the summary-statistics definitions (oracle/summary.py) on
trajectories whose answers are known in closed form."""
import numpy as np

from oracle import summary


def _traj(positions, L=(50.0, 50.0), vol=100, surf=40):
    """positions: (K, ncells, 2) -> V, S, pos arrays with a medium entry 0."""
    pos = np.asarray(positions, dtype=np.float64)
    K, C, _ = pos.shape
    V = np.full((K, C + 1), vol, dtype=np.float64)
    S = np.full((K, C + 1), surf, dtype=np.float64)
    V[:, 0] = 0
    P = np.zeros((K, C + 1, 2))
    P[:, 1:, :] = np.mod(pos, np.asarray(L))
    return V, S, P


def test_constant_velocity():
    K = 12
    pos = np.array([[[3.0 + 2.0 * k, 5.0 + 1.5 * k]] for k in range(K)])  # crosses x = 50
    V, S, P = _traj(pos)
    out = summary.summary(V, S, P, (50, 50), interval=10.0)
    assert np.isclose(out[0], 100) and out[1] == 0
    assert np.isclose(out[2], 40) and out[3] == 0
    assert np.isclose(out[4], np.hypot(2.0, 1.5) / 10.0)
    assert out[5] < 1e-20
    # directions never decorrelate: persistence is the longest lag, K - 2 steps
    assert np.isclose(out[6], (K - 2) * 10.0)


def test_alternating_direction():
    K = 9
    pos = np.array([[[10.0 + (k % 2) * 3.0, 10.0]] for k in range(K)])
    V, S, P = _traj(pos)
    out = summary.summary(V, S, P, (50, 50), interval=5.0)
    assert np.isclose(out[4], 3.0 / 5.0)
    # A(1) = -1: interpolated crossing at (1 - 1/e) / 2 of the first lag
    assert np.isclose(out[6], 5.0 * (1 - np.exp(-1)) / 2.0)


def test_persistence_interpolates_from_the_last_defined_lag():
    # the cell moves +x, rests, moves -x, rests, moves +x: no lag-1 pair of
    # unit steps is defined (every pair holds a rest), lag 2 pairs are
    # (+x, -x) and (-x, +x), so A(2) = -1 and A(1) is undefined; the 1/e
    # crossing lies on the line from A(0) = 1 to A(2) = -1:
    # tau = 2 (1 - 1/e) / 2 = 1 - 1/e sample intervals
    xs = [10.0, 13.0, 13.0, 10.0, 10.0, 13.0]
    pos = np.array([[[x, 20.0]] for x in xs])
    V, S, P = _traj(pos)
    out = summary.summary(V, S, P, (50, 50), interval=4.0)
    assert np.isclose(out[6], 4.0 * (1.0 - np.exp(-1.0)))
    assert out[7] == 0.0


def test_minimum_image_and_dead_cells():
    # a jump from x = 49 to x = 1 is a step of +2 on a 50-periodic axis
    pos = np.array([[[49.0, 0.0], [10.0, 10.0]], [[1.0, 0.0], [10.0, 10.0]], [[3.0, 0.0], [12.0, 10.0]]])
    V, S, P = _traj(pos)
    V[1, 2] = 0  # cell 2 dead at the middle sample
    out = summary.summary(V, S, P, (50, 50), interval=1.0)
    # speeds: cell 1 two steps of 2; cell 2 has no pair alive at both ends
    assert np.isclose(out[4], 2.0) and out[5] < 1e-20
    # volumes: five alive (cell, sample) pairs of 100
    assert np.isclose(out[0], 100.0)


def test_volume_variance_closed_form():
    rng = np.random.default_rng(0)
    K, C = 7, 5
    V = np.zeros((K, C + 1))
    V[:, 1:] = rng.integers(50, 150, size=(K, C))
    S = V * 0.5
    P = np.zeros((K, C + 1, 2))
    out = summary.summary(V, S, P, (30, 30), interval=1.0)
    vals = V[:, 1:].ravel()
    assert np.isclose(out[0], vals.mean()) and np.isclose(out[1], ((vals - vals.mean()) ** 2).mean())
    assert np.isclose(out[2], 0.5 * vals.mean()) and np.isclose(out[3], 0.25 * ((vals - vals.mean()) ** 2).mean())


def test_random_directions_decorrelate_at_first_lag():
    rng = np.random.default_rng(1)
    K, C = 60, 40
    ang = rng.uniform(0, 2 * np.pi, size=(K - 1, C))
    steps = np.stack([np.cos(ang), np.sin(ang)], axis=-1)
    pos = np.concatenate([np.zeros((1, C, 2)), np.cumsum(steps, axis=0)], axis=0) + 20.0
    V, S, P = _traj(pos, L=(1000.0, 1000.0))
    out = summary.summary(V, S, P, (1000, 1000), interval=1.0)
    assert np.isclose(out[4], 1.0)
    # A(1) ~ 0, so persistence ~ (1 - 1/e) / (1 - 0) of one lag
    assert abs(out[6] - (1 - np.exp(-1))) < 0.1


def _track(steps, L=100.0):
    # one cell moving by the given 2D steps from (10, 10); V = 50 throughout
    p = [np.array([10.0, 10.0])]
    for s_ in steps:
        p.append(np.mod(p[-1] + np.asarray(s_, dtype=np.float64), L))
    K = len(p)
    pos = np.zeros((K, 2, 2))
    pos[:, 1, :] = np.asarray(p)
    V = np.zeros((K, 2))
    V[:, 1] = 50
    return V, pos


def test_autocorrelation_closed_forms():
    # straight line: A = 1 at every lag; reversals: (-1)^tau; right-angle turns
    # every step: 1, 0, -1, 0, ...; across the periodic boundary too
    V, pos = _track([(3, 0)] * 6)
    s, n = summary.autocorrelation(V, pos, (100, 100))
    assert np.allclose(s / n, 1.0) and list(n) == [6, 5, 4, 3, 2, 1]
    V, pos = _track([(2, 0), (-2, 0)] * 3)
    s, n = summary.autocorrelation(V, pos, (100, 100))
    assert np.allclose(s / n, [(-1) ** t for t in range(6)])
    V, pos = _track([(0, 1), (-1, 0), (0, -1), (1, 0)] * 2)
    s, n = summary.autocorrelation(V, pos, (100, 100))
    assert np.allclose(s / n, [1, 0, -1, 0, 1, 0, -1, 0][:8])
    V, pos = _track([(30, 0)] * 5, L=100.0)  # wraps around x twice
    s, n = summary.autocorrelation(V, pos, (100, 100))
    assert np.allclose(s / n, 1.0)


def test_autocorrelation_skips_dead_and_still_cells():
    V, pos = _track([(1, 0), (0, 0), (1, 0), (1, 0)])  # step 1 has no direction
    s, n = summary.autocorrelation(V, pos, (100, 100))
    assert list(n) == [3, 1, 1, 1] and np.allclose(s / n, 1.0)
    V[2, 1] = 0  # dead at sample 2: steps 1 and 2 undefined
    s, n = summary.autocorrelation(V, pos, (100, 100))
    assert list(n) == [2, 0, 0, 1]


def test_autocorrelation_of_a_random_walk_decays():
    rng = np.random.Generator(np.random.PCG64(4))
    ang = rng.uniform(0, 2 * np.pi, 1200)
    V, pos = _track(np.stack([np.cos(ang), np.sin(ang)], 1) * 2.0, L=1e9)
    s, n = summary.autocorrelation(V, pos, (1e9, 1e9))
    a = s / n
    assert a[0] == 1.0 and np.all(np.abs(a[1:20]) < 0.1)
