"""Distribution pins of the oracle's Markov chains on lattices small enough to
enumerate every state.

For a single cell on a medium background (two labels), the test builds the
exact transition operator of each chain from the paper's definitions, using
its own full Hamiltonian (eq. 1 + eq. 3) and the Metropolis rule (eq. 2):

* serial CPM (Methods): a uniform site copies from a uniform Moore neighbour;
* the deterministic checkerboard scheme: in each activation every thread area
  makes one attempt in the active sub-area, all attempts of an activation see
  the state of the activation start, colours take turns;
* the symmetric proposal, whose stationary law is the Boltzmann distribution.

It propagates the initial state exactly for a few MCS and compares the law
with the final states of many independent oracle runs (chi-square test).  A
dropped energy term, a wrong sign, a wrong neighbour list, a wrong target
mapping or a wrong visibility rule changes the law and fails these tests.
"""
import numpy as np
import pytest
from scipy import stats

import oracle

J_CM = 2.0
LAM_V, V_T = 1.0, 4
LAM_S, S_T = 0.25, 16
T = 2.5


def _model(dims, s=1, k=1):
    J = np.array([[0.0, J_CM], [J_CM, 0.0]])
    return oracle.Model(2, dims, J, [0.0, LAM_V], [0, V_T], [0.0, LAM_S], [0, S_T], T=T, s=s, k=k,
                        seed=12345)


def _moore2():
    return [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]


def _all_states(Ly, Lx):
    N = Ly * Lx
    idx = np.arange(2 ** N)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1  # site i = x + Lx*y is bit i
    return bits.reshape(-1, Ly, Lx)


def _energy(states):
    """Full H of every two-label state (label 1 = the cell, 0 = medium)."""
    adh = np.zeros(len(states))
    S = np.zeros(len(states))
    for dy, dx in _moore2():
        nb = np.roll(states, shift=(-dy, -dx), axis=(1, 2))
        unlike = states != nb
        adh += unlike.sum(axis=(1, 2)) * J_CM
        S += (unlike & (states == 1)).sum(axis=(1, 2))
    V = states.sum(axis=(1, 2))
    # the cell keeps its constraint terms at zero volume: the sum of eq. 1
    # runs over cells, and the local energy change of removing the last site
    # is that of V: 1 -> 0
    return adh / 2 + LAM_V * (V - V_T) ** 2 + LAM_S * (S - S_T) ** 2


def _acc(dh):
    return np.where(dh <= 0, 1.0, np.exp(-np.maximum(dh, 0) / T))


def _flip_prob_neighbour(states, H, t, Lx):
    """Probability that a copy attempt at site t (from a uniform Moore
    neighbour) flips t, for every state."""
    Ly = states.shape[1]
    y, x = divmod(t, Lx)
    lab = states[:, y, x]
    unlike = np.zeros(len(states))
    for dy, dx in _moore2():
        unlike += states[:, (y + dy) % Ly, (x + dx) % Lx] != lab
    idx = np.arange(len(states))
    dh = H[idx ^ (1 << t)] - H
    return unlike / 8.0 * _acc(dh)


def _states_to_index(lats):
    N = lats.shape[1]
    return (lats.astype(np.int64) << np.arange(N)[None, :]).sum(axis=1)


def _chi2_pvalue(counts, expected):
    # pool bins with small expectation into one
    small = expected < 5
    obs = np.concatenate([counts[~small], [counts[small].sum()]])
    exp = np.concatenate([expected[~small], [expected[small].sum()]])
    keep = exp > 0
    obs, exp = obs[keep], exp[keep]
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    return stats.chi2.sf(chi2, len(obs) - 1)


def test_dcs_law_2x4_s1():
    Ly, Lx = 2, 4
    states = _all_states(Ly, Lx)
    H = _energy(states)
    N = Ly * Lx
    init = np.zeros((Ly, Lx), dtype=np.int32)
    init[:, :2] = 1
    p = np.zeros(2 ** N)
    p[_states_to_index(init.reshape(1, -1))[0]] = 1.0
    n_mcs = 3
    idx = np.arange(2 ** N)
    for _ in range(n_mcs):
        for alpha in range(4):  # (2s)^d / k = 4 activations, colour = alpha
            cx, cy = alpha & 1, (alpha >> 1) & 1
            active = [(2 * ay + cy) * Lx + (2 * ax + cx) for ay in range(Ly // 2) for ax in range(Lx // 2)]
            f = [_flip_prob_neighbour(states, H, t, Lx) for t in active]
            new = np.zeros_like(p)
            for mask in range(2 ** len(active)):
                w = np.ones(2 ** N)
                flip = 0
                for b, t in enumerate(active):
                    if mask >> b & 1:
                        w = w * f[b]
                        flip |= 1 << t
                    else:
                        w = w * (1 - f[b])
                np.add.at(new, idx ^ flip, p * w)
            p = new
    assert abs(p.sum() - 1) < 1e-12
    R = 200000
    finals = oracle.replicates(_model((Lx, Ly), s=1), init, [0, 1], n_mcs, R, "dcs")
    counts = np.bincount(_states_to_index(finals), minlength=2 ** N)
    assert _chi2_pvalue(counts, p * R) > 1e-4


def test_dcs_law_4x4_s2():
    # one thread area; each activation one attempt at a uniform site of the
    # active 2x2 sub-area (16 activations per MCS, colour = alpha mod 4)
    Ly, Lx = 4, 4
    states = _all_states(Ly, Lx)
    H = _energy(states)
    N = Ly * Lx
    init = np.zeros((Ly, Lx), dtype=np.int32)
    init[1:3, 1:3] = 1
    p = np.zeros(2 ** N)
    p[_states_to_index(init.reshape(1, -1))[0]] = 1.0
    idx = np.arange(2 ** N)
    f_all = [_flip_prob_neighbour(states, H, t, Lx) for t in range(N)]
    n_mcs = 2
    for _ in range(n_mcs):
        for alpha in range(16):
            cx, cy = alpha % 4 & 1, (alpha % 4 >> 1) & 1
            sub = [(2 * cy + oy) * Lx + (2 * cx + ox) for oy in range(2) for ox in range(2)]
            new = np.zeros_like(p)
            stay = np.ones(2 ** N)
            for t in sub:
                ft = f_all[t] / 4.0
                np.add.at(new, idx ^ (1 << t), p * ft)
                stay -= ft
            new += p * stay
            p = new
    R = 200000
    finals = oracle.replicates(_model((Lx, Ly), s=2), init, [0, 1], n_mcs, R, "dcs")
    # compare the law of the macrostate (V, S) and of the full state
    fidx = _states_to_index(finals)
    counts = np.bincount(fidx, minlength=2 ** N)
    assert _chi2_pvalue(counts, p * R) > 1e-4
    V = states.sum(axis=(1, 2))
    macro_p = np.bincount(V, weights=p, minlength=N + 1)
    macro_c = np.bincount(V[fidx], minlength=N + 1)
    assert _chi2_pvalue(macro_c, macro_p * R) > 1e-4


def test_serial_law_3x3():
    Ly, Lx = 3, 3
    states = _all_states(Ly, Lx)
    H = _energy(states)
    N = Ly * Lx
    init = np.zeros((Ly, Lx), dtype=np.int32)
    init[0:2, 0:2] = 1
    p = np.zeros(2 ** N)
    p[_states_to_index(init.reshape(1, -1))[0]] = 1.0
    idx = np.arange(2 ** N)
    f_all = [_flip_prob_neighbour(states, H, t, Lx) / N for t in range(N)]
    n_mcs = 2
    for _ in range(n_mcs * N):
        new = np.zeros_like(p)
        stay = np.ones(2 ** N)
        for t in range(N):
            np.add.at(new, idx ^ (1 << t), p * f_all[t])
            stay -= f_all[t]
        p = new + p * stay
    R = 200000
    m = oracle.Model(2, (Lx, Ly), [[0, J_CM], [J_CM, 0]], [0, LAM_V], [0, V_T], [0, LAM_S], [0, S_T],
                     T=T, seed=99)
    finals = oracle.replicates(m, init, [0, 1], n_mcs, R, "serial")
    counts = np.bincount(_states_to_index(finals), minlength=2 ** N)
    assert _chi2_pvalue(counts, p * R) > 1e-4


def test_symmetric_proposal_reaches_boltzmann():
    # with a symmetric proposal the Metropolis rule of eq. 2 leaves exp(-H/T)
    # invariant: after many sweeps the law of the state is the Boltzmann law
    Ly, Lx = 3, 3
    states = _all_states(Ly, Lx)
    H = _energy(states)
    N = Ly * Lx
    boltz = np.exp(-(H - H.min()) / T)
    boltz /= boltz.sum()
    # exact propagation for the finite-time check
    idx = np.arange(2 ** N)
    f_all = [_acc(H[idx ^ (1 << t)] - H) / N for t in range(N)]
    init = np.zeros((Ly, Lx), dtype=np.int32)
    init[1, :] = 1
    p = np.zeros(2 ** N)
    p[_states_to_index(init.reshape(1, -1))[0]] = 1.0
    n_mcs = 40
    for _ in range(n_mcs * N):
        new = np.zeros_like(p)
        stay = np.ones(2 ** N)
        for t in range(N):
            np.add.at(new, idx ^ (1 << t), p * f_all[t])
            stay -= f_all[t]
        p = new + p * stay
    assert 0.5 * np.abs(p - boltz).sum() < 1e-3  # the chain has mixed
    R = 100000
    m = oracle.Model(2, (Lx, Ly), [[0, J_CM], [J_CM, 0]], [0, LAM_V], [0, V_T], [0, LAM_S], [0, S_T],
                     T=T, seed=5)
    finals = oracle.replicates(m, init, [0, 1], n_mcs, R, "symmetric")
    counts = np.bincount(_states_to_index(finals), minlength=2 ** N)
    assert _chi2_pvalue(counts, boltz * R) > 1e-4
    assert _chi2_pvalue(counts, p * R) > 1e-4


@pytest.mark.parametrize("wrong", ["no_surface", "double_J"])
def test_chain_test_has_power(wrong):
    # the DCS law check rejects a model that differs in one term
    Ly, Lx = 2, 4
    N = Ly * Lx
    init = np.zeros((Ly, Lx), dtype=np.int32)
    init[:, :2] = 1
    states = _all_states(Ly, Lx)
    H = _energy(states)
    idx = np.arange(2 ** N)
    p = np.zeros(2 ** N)
    p[_states_to_index(init.reshape(1, -1))[0]] = 1.0
    for _ in range(3):
        for alpha in range(4):
            cx, cy = alpha & 1, (alpha >> 1) & 1
            active = [(2 * ay + cy) * Lx + (2 * ax + cx) for ay in range(Ly // 2) for ax in range(Lx // 2)]
            f = [_flip_prob_neighbour(states, H, t, Lx) for t in active]
            new = np.zeros_like(p)
            for mask in range(4):
                w = np.ones(2 ** N)
                flip = 0
                for b, t in enumerate(active):
                    w = w * (f[b] if mask >> b & 1 else 1 - f[b])
                    flip |= (1 << t) if mask >> b & 1 else 0
                np.add.at(new, idx ^ flip, p * w)
            p = new
    J = np.array([[0.0, J_CM], [J_CM, 0.0]]) * (2 if wrong == "double_J" else 1)
    ls = [0.0, 0.0] if wrong == "no_surface" else [0.0, LAM_S]
    m = oracle.Model(2, (Lx, Ly), J, [0.0, LAM_V], [0, V_T], ls, [0, S_T], T=T, s=1, seed=12345)
    R = 200000
    finals = oracle.replicates(m, init, [0, 1], 3, R, "dcs")
    counts = np.bincount(_states_to_index(finals), minlength=2 ** N)
    assert _chi2_pvalue(counts, p * R) < 1e-6
