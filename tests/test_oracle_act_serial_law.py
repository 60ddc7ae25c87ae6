"""Exact-law pin of the serial CPM (Methods, first paragraph) with the Act
term (eq. 7 and eq. 8): the reference that the parallel scheme's
polarisation runs are compared with.

A 3x3 periodic lattice, one motile cell of four sites on medium, Max_act 3
with starting activities 3 and 1.  An MCS is 9 attempts, each at a uniform
site, copying from a uniform Moore neighbour, every attempt seeing the
lattice, counters and activities that the previous one left.  The state is
(labels, activities), and its law after one MCS is propagated from the
definitions (H from eq. 1 and eq. 3; Delta H_act = R (GM(t) - GM(s)),
R = lambda_act / Max_act, GM the geometric mean of the activities of a site
and its Moore neighbours in the same cell, 0 for medium or a zero factor;
activity Max_act on a copy by the cell, 0 on a copy by medium; decay by one
at the end of the MCS; Metropolis acceptance in float64).  Oracle runs are
compared with it by a chi-square test; the laws without the Act term or with
its sign flipped are rejected by the same samples.
"""
import numpy as np
import pytest
from scipy import stats

import oracle

L = 3
N = L * L
J_CM = 2.0
LAM_V, V_T = 1.0, 4
LAM_S, S_T = 0.25, 16
LAM_ACT, MAX_ACT = 6.0, 3
T = 2.5
R_REP = 200000
_NB = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]


def _site(y, x):
    return (y % L) * L + (x % L)


_NBR = np.array([[_site(i // L + dy, i % L + dx) for dy, dx in [(0, 0)] + _NB] for i in range(N)])


def _h_table():
    idx = np.arange(2 ** N)
    lab = ((idx[:, None] >> np.arange(N)[None, :]) & 1).reshape(-1, L, L)
    adh = np.zeros(len(lab))
    S = np.zeros(len(lab))
    for dy, dx in _NB:
        nb = np.roll(lab, shift=(-dy, -dx), axis=(1, 2))
        unlike = lab != nb
        adh += unlike.sum(axis=(1, 2)) * J_CM
        S += (unlike & (lab == 1)).sum(axis=(1, 2))
    V = lab.sum(axis=(1, 2))
    return adh / 2 + LAM_V * (V - V_T) ** 2 + LAM_S * (S - S_T) ** 2


def _decode(keys):
    lab = ((keys[:, None] >> np.arange(N)[None, :]) & 1).astype(np.int64)
    act = ((keys[:, None] >> (N + 2 * np.arange(N))[None, :]) & 3).astype(np.int64)
    return lab, act


def _encode(lab, act):
    sh = np.arange(N)[None, :]
    return ((lab << sh).sum(axis=1) | (act << (N + 2 * sh)).sum(axis=1)).astype(np.int64)


def _gm(lab, act):
    own = lab[:, _NBR]
    a = act[:, _NBR].astype(np.float64)
    member = own == lab[:, :, None]
    cnt = member.sum(axis=2)
    zero = (member & (a == 0)).any(axis=2)
    la = np.where(member & (a > 0), np.log(np.where(a > 0, a, 1.0)), 0.0)
    g = np.where(zero, 0.0, np.exp(la.sum(axis=2) / cnt))
    return np.where(lab == 1, g, 0.0)


def _merge(keys, w):
    u, inv = np.unique(keys, return_inverse=True)
    p = np.bincount(inv.reshape(-1), weights=w)
    keep = p > 0
    return u[keep], p[keep]


def _initial():
    lab = np.zeros((L, L), dtype=np.int64)
    lab[0:2, 0:2] = 1
    act = np.zeros((L, L), dtype=np.int64)
    act[0:2, 0:2] = [[3, 1], [1, 3]]
    return lab, act


def _law(H, variant=None):
    R = LAM_ACT / MAX_ACT
    lab0, act0 = _initial()
    keys = _encode(lab0.reshape(1, -1), act0.reshape(1, -1))
    p = np.ones(1)
    sh = np.arange(N)[None, :]
    for _ in range(N):
        lab, act = _decode(keys)
        hk = H[(lab << sh).sum(axis=1)]
        gm = _gm(lab, act)
        out_k, out_w = [keys], [p.copy()]
        for t in range(N):
            for n in range(1, 9):
                s = _NBR[t, n]
                move = lab[:, t] != lab[:, s]
                nl = lab.copy()
                nl[:, t] = lab[:, s]
                na = act.copy()
                na[:, t] = np.where(lab[:, s] == 1, MAX_ACT, 0)
                dh = H[(nl << sh).sum(axis=1)] - hk
                if variant != "no_act":
                    sign = -1.0 if variant == "flipped" else 1.0
                    dh = dh + sign * R * (gm[:, t] - gm[:, s])
                acc = np.where(dh <= 0, 1.0, np.exp(-np.maximum(dh, 0.0) / T))
                f = np.where(move, acc, 0.0) * p / (8.0 * N)
                out_k.append(_encode(nl, na))
                out_w.append(f)
                out_w[0] -= f
        keys, p = _merge(np.concatenate(out_k), np.concatenate(out_w))
    lab, act = _decode(keys)
    return _merge(_encode(lab, np.maximum(act - 1, 0)), p)


def _chi2_pvalue(counts, expected):
    small = expected < 5
    obs = np.concatenate([counts[~small], [counts[small].sum()]])
    exp = np.concatenate([expected[~small], [expected[small].sum()]])
    keep = exp > 0
    obs, exp = obs[keep], exp[keep]
    return stats.chi2.sf(float(np.sum((obs - exp) ** 2 / exp)), len(obs) - 1)


def _counts(keys, law_keys):
    pos = np.minimum(np.searchsorted(law_keys, keys), len(law_keys) - 1)
    inside = law_keys[pos] == keys
    return np.bincount(pos[inside], minlength=len(law_keys)), int((~inside).sum())


@pytest.fixture(scope="module")
def runs():
    lab, act = _initial()
    m = oracle.Model(2, (L, L), [[0.0, J_CM], [J_CM, 0.0]], [0.0, LAM_V], [0, V_T], [0.0, LAM_S], [0, S_T],
                     lambda_act=[0.0, LAM_ACT], max_act=[0, MAX_ACT], T=T, seed=8080)
    fl = np.zeros((R_REP, N), dtype=np.int64)
    fa = np.zeros((R_REP, N), dtype=np.int64)
    for r in range(R_REP):
        m.c.lattice_id = r
        st = oracle.State(m, lab, [0, 1], act)
        st.serial_sweep(1)
        fl[r], fa[r] = st.lattice, st.act
    return _encode(fl, fa)


@pytest.fixture(scope="module")
def table():
    return _h_table()


def test_serial_act_law(runs, table):
    k, p = _law(table)
    assert abs(p.sum() - 1.0) < 1e-9
    counts, outside = _counts(runs, k)
    assert outside == 0
    assert _chi2_pvalue(counts, p * R_REP) > 1e-4


@pytest.mark.parametrize("variant", ["no_act", "flipped"])
def test_serial_act_law_has_power(runs, table, variant):
    k, p = _law(table, variant)
    counts, outside = _counts(runs, k)
    assert outside > 0 or _chi2_pvalue(counts, p * R_REP) < 1e-6
