"""Exact-law pin of the persistence term (Methods, eq. 5) under the parallel
scheme, on a 4x4 lattice where every label pattern can be enumerated.

One cell on medium, sub-area edge s = 2 (one thread area, 16 activations per
MCS).  The cell's direction changes only at the end of an MCS (eq. 6), so
within the first MCS it is the one it starts with, and the chain lives on the
2^16 label patterns.  Its law after one MCS is propagated from the
definitions: H from eq. 1 and eq. 3 (the full Hamiltonian of the chain
tests); a copy by the cell from source i into target j adds
-lambda_P * (unit(j - i) . P), P the cell's direction (read so that copies
along it are favoured); medium copies add nothing; Metropolis acceptance
(eq. 2), float64.  Oracle runs that start from the same direction are
compared with it by a chi-square test, and laws without the term, with its
sign flipped, or with the direction's components swapped are rejected by the
same samples.
"""
import numpy as np
import pytest

import oracle
from tests.test_oracle_chain import (J_CM, LAM_S, LAM_V, S_T, T, V_T, _all_states, _chi2_pvalue, _energy,
                                     _states_to_index)

L = 4
N = L * L
LAM_P = 4.0
R_REP = 100000
_NB = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]
# the starting direction: unit vector at 30 degrees, in units of 2^-14
P0 = np.array([np.rint(16384 * np.cos(np.pi / 6)), np.rint(16384 * np.sin(np.pi / 6)), 0], dtype=np.int32)


def _initial():
    init = np.zeros((L, L), dtype=np.int32)
    init[1:3, 1:3] = 1
    return init


def _law(variant=None):
    states = _all_states(L, L)
    H = _energy(states)
    lab = states.reshape(len(states), -1)
    P = P0[:2].astype(np.float64) / 16384.0
    if variant == "swapped":
        P = P[::-1]
    idx = np.arange(2 ** N)
    p = np.zeros(2 ** N)
    p[_states_to_index(_initial().reshape(1, -1))[0]] = 1.0
    flip = {}
    for t in range(N):
        ty, tx = divmod(t, L)
        for dy, dx in _NB:
            s = ((ty + dy) % L) * L + (tx + dx) % L
            move = lab[:, t] != lab[:, s]
            dh = H[idx ^ (1 << t)] - H
            u = np.array([-dx, -dy], dtype=np.float64) / np.hypot(dx, dy)   # unit vector source -> target
            term = -LAM_P * float(u @ P)
            if variant == "flipped":
                term = -term
            if variant != "no_term":
                dh = dh + np.where(lab[:, s] == 1, term, 0.0)
            acc = np.where(dh <= 0, 1.0, np.exp(-np.maximum(dh, 0.0) / T))
            flip[(t, dy, dx)] = np.where(move, acc, 0.0) / 32.0
    for alpha in range(16):
        phi = alpha % 4
        cx, cy = phi & 1, (phi >> 1) & 1
        new = np.zeros_like(p)
        stay = np.ones(2 ** N)
        for oy in range(2):
            for ox in range(2):
                t = (2 * cy + oy) * L + 2 * cx + ox
                for dy, dx in _NB:
                    f = flip[(t, dy, dx)]
                    np.add.at(new, idx ^ (1 << t), p * f)
                    stay -= f
        p = new + p * stay
    return p


@pytest.fixture(scope="module")
def counts():
    m = oracle.Model(2, (L, L), [[0.0, J_CM], [J_CM, 0.0]], [0.0, LAM_V], [0, V_T], [0.0, LAM_S], [0, S_T],
                     T=T, s=2, k=1, seed=4242, lambda_P=[0.0, LAM_P], mu_P=[0.0, 0.5], dt_P=1)
    init = _initial()
    finals = np.zeros((R_REP, N), dtype=np.int32)
    for r in range(R_REP):
        m.c.lattice_id = r
        st = oracle.State(m, init, [0, 1])
        st.P[3:6] = P0
        st.sweep(1)
        finals[r] = st.lattice
    return np.bincount(_states_to_index(finals), minlength=2 ** N)


def test_persistence_law(counts):
    p = _law()
    assert abs(p.sum() - 1.0) < 1e-9
    assert _chi2_pvalue(counts, p * R_REP) > 1e-4


@pytest.mark.parametrize("variant", ["no_term", "flipped", "swapped"])
def test_persistence_law_has_power(counts, variant):
    assert _chi2_pvalue(counts, _law(variant) * R_REP) < 1e-6
