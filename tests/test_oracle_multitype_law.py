"""Exact-law pin of a multi-type model under the parallel scheme with two
thread areas working at once (Results, parallel scheme; Methods, eq. 1-3).

A 2x4 periodic lattice with sub-area edge s = 1 holds two thread areas; in
each of the 4 activations of an MCS both make one attempt, at the site of
the active colour, and both attempts read the cell sizes and surfaces as
they stood when the activation began (the two targets are not neighbours,
so neither reads the site the other writes).  Three labels, medium and two
cells whose types differ from their labels (cell 1 has type 2, cell 2 type
1), with a type-dependent J, volume and surface constraint: all 3^8 label
patterns are enumerated and the law after three MCS is propagated from the
full Hamiltonian and the Metropolis rule.  Oracle runs are compared with it
by a chi-square test; the same samples reject the law built with the types
taken from the labels, and the law in which the second attempt of an
activation sees the first one's result.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle

LX, LY = 4, 2
N = LX * LY
J = np.array([[0.0, 2.0, 3.0], [2.0, 4.0, 1.0], [3.0, 1.0, 5.0]])   # by type: medium, 1, 2
LAM_V = np.array([0.0, 1.0, 0.5])
V_T = np.array([0, 2, 4])
LAM_S = np.array([0.0, 0.25, 0.125])
S_T = np.array([0, 10, 12])
T = 3.0
CELL_TYPE = np.array([0, 2, 1], dtype=np.int32)
N_MCS = 3
R_REP = 200000
_NB = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]


def _states():
    return np.array(list(itertools.product(range(3), repeat=N)), dtype=np.int64)[:, ::-1]  # site i = digit i


def _index(lab):
    return (lab * (3 ** np.arange(N))[None, :]).sum(axis=1)


def _energy(states, types):
    lab = states.reshape(-1, LY, LX)
    tau = types[lab]
    H = np.zeros(len(states))
    S = np.zeros((len(states), 3))
    for dy, dx in _NB:
        nb = np.roll(lab, shift=(-dy, -dx), axis=(1, 2))
        unlike = lab != nb
        H += (J[tau, types[nb]] * unlike).sum(axis=(1, 2)) / 2
        for c in (1, 2):
            S[:, c] += (unlike & (lab == c)).sum(axis=(1, 2))
    for c in (1, 2):
        tc = types[c]
        V = (lab == c).sum(axis=(1, 2))
        H += LAM_V[tc] * (V - V_T[tc]) ** 2 + LAM_S[tc] * (S[:, c] - S_T[tc]) ** 2
    return H


def _moves(states, H, t):
    """Per state, the probability that an attempt at t ends with each label."""
    y, x = divmod(t, LX)
    P = np.zeros((len(states), 3))
    cur = states[:, t]
    for dy, dx in _NB:
        s = ((y + dy) % LY) * LX + (x + dx) % LX
        nl = states[:, s]
        new = states.copy()
        new[:, t] = nl
        dh = H[_index(new)] - H
        acc = np.where(dh <= 0, 1.0, np.exp(-np.maximum(dh, 0.0) / T))
        P[np.arange(len(states)), nl] += np.where(nl != cur, acc, 0.0) / 8.0
    P[np.arange(len(states)), cur] += 1.0 - P.sum(axis=1)
    return P


def _initial():
    lab = np.zeros((LY, LX), dtype=np.int64)
    lab[:, 0:2] = 1
    lab[:, 2] = 2
    return lab


def _law(types, sequential=False):
    states = _states()
    H = _energy(states, types)
    p = np.zeros(len(states))
    p[_index(_initial().reshape(1, -1))[0]] = 1.0
    pow3 = 3 ** np.arange(N)
    for _ in range(N_MCS):
        for alpha in range(4):
            cx, cy = alpha & 1, (alpha >> 1) & 1
            sites = [cy * LX + cx, cy * LX + 2 + cx]
            if sequential:
                for t in sites:
                    P = _moves(states, H, t)
                    new = np.zeros_like(p)
                    for lbl in range(3):
                        dest = _index(states) + (lbl - states[:, t]) * pow3[t]
                        np.add.at(new, dest, p * P[:, lbl])
                    p = new
                continue
            Pa, Pb = _moves(states, H, sites[0]), _moves(states, H, sites[1])
            new = np.zeros_like(p)
            for la in range(3):
                for lb in range(3):
                    dest = (_index(states) + (la - states[:, sites[0]]) * pow3[sites[0]]
                            + (lb - states[:, sites[1]]) * pow3[sites[1]])
                    np.add.at(new, dest, p * Pa[:, la] * Pb[:, lb])
            p = new
    return p


def _chi2_pvalue(counts, expected):
    small = expected < 5
    obs = np.concatenate([counts[~small], [counts[small].sum()]])
    exp = np.concatenate([expected[~small], [expected[small].sum()]])
    keep = exp > 0
    obs, exp = obs[keep], exp[keep]
    return stats.chi2.sf(float(np.sum((obs - exp) ** 2 / exp)), len(obs) - 1)


@pytest.fixture(scope="module")
def counts():
    m = oracle.Model(2, (LX, LY), J, LAM_V, V_T, LAM_S, S_T, T=T, s=1, k=1, seed=606)
    finals = oracle.replicates(m, _initial().astype(np.int32), CELL_TYPE, N_MCS, R_REP, "dcs")
    return np.bincount(_index(finals.astype(np.int64)), minlength=3 ** N)


def test_multitype_law(counts):
    p = _law(CELL_TYPE)
    assert abs(p.sum() - 1.0) < 1e-9
    assert _chi2_pvalue(counts, p * R_REP) > 1e-4


@pytest.mark.parametrize("wrong", ["types_from_labels", "sequential"])
def test_multitype_law_has_power(counts, wrong):
    if wrong == "types_from_labels":
        p = _law(np.array([0, 1, 2]))
    else:
        p = _law(CELL_TYPE, sequential=True)
    assert _chi2_pvalue(counts, p * R_REP) < 1e-6
