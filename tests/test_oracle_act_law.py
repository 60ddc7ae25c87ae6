"""Exact-law pin of the Act extension (Methods, eq. 7 and eq. 8) under the
parallel scheme, on a lattice small enough to enumerate every reachable state.

A single motile cell on medium, 4x4 periodic lattice, sub-area edge s = 2, so
one thread area and 16 activations per MCS: activation alpha has colour
alpha mod 4 and makes one copy attempt at a uniform site of its 2x2 sub-area,
from a uniform Moore neighbour.  The state is the label of every site and the
activity of every cell site, so the chain is Markov and its law can be
propagated exactly, from the definitions written out here:

* H (eq. 1 and eq. 3): adhesion over unlike Moore pairs, volume and surface
  constraints, tabulated for all 2^16 label patterns;
* Delta H_act = R * (GM(t) - GM(s)) with R = lambda_act / Max_act (eq. 7,
  read so that copies out of active regions are favoured), where GM(x) is the
  geometric mean of the activities of x and its Moore neighbours that belong
  to x's cell, 0 for medium or when one of them is 0 (eq. 8);
* Metropolis acceptance (eq. 2), in float64;
* an accepted copy sets the target's activity to Max_act when the copying
  label is the cell, to 0 when it is medium; every activity drops by one (not
  below 0) at the end of each MCS.

The law after one MCS (135,424 reachable states; a second MCS would take
millions) is compared with the final (label, activity) states of many
independent oracle runs by a chi-square test.  The cell starts with mixed
activities (Max_act = 3 and 1), so geometric means differ from arithmetic
ones from the first attempt on, and the final states carry the decay.  Laws
built with the Act term dropped, with its sign flipped, with an arithmetic
mean for GM, with GM over every neighbour regardless of label, or without
decay are rejected by the same samples (p below 1e-100 for each), so a
mistake of that kind in the oracle would fail here.  With k = 4 attempts per
activation (each area's attempts back to back, seeing its own deltas) the
law is pinned the same way, and the k = 1 law is rejected by those samples.
The oracle's fixed-point energies differ from these float64 ones by far less
than the test can resolve.
"""
import numpy as np
import pytest
from scipy import stats

import oracle

L = 4
N = L * L
J_CM = 2.0
LAM_V, V_T = 1.0, 4
LAM_S, S_T = 0.25, 16
LAM_ACT, MAX_ACT = 6.0, 3
T = 2.5
N_MCS = 1
R_REP = 200000

_NB = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx]


def _site(y, x):
    return (y % L) * L + (x % L)


# Moore neighbours of every site, and the site itself first
_NBR = np.array([[_site(i // L + dy, i % L + dx) for dy, dx in [(0, 0)] + _NB] for i in range(N)])


def _h_table():
    """Full H (eq. 1 + eq. 3) of every label pattern; bit i is site i."""
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


def _gm(lab, act, variant):
    """GM of every site of every state (eq. 8), as an (M, N) float64 array."""
    own = lab[:, _NBR]                      # (M, N, 9) labels of x and its neighbours
    a = act[:, _NBR].astype(np.float64)
    if variant == "all_neighbours":
        member = np.ones_like(own, dtype=bool)
    else:
        member = own == lab[:, :, None]
    cnt = member.sum(axis=2)
    if variant == "arithmetic":
        g = np.where(member, a, 0.0).sum(axis=2) / cnt
    else:
        zero = (member & (a == 0)).any(axis=2)
        with np.errstate(divide="ignore"):
            la = np.where(member & (a > 0), np.log(np.where(a > 0, a, 1.0)), 0.0)
        g = np.where(zero, 0.0, np.exp(la.sum(axis=2) / cnt))
    return np.where(lab == 1, g, 0.0)


def _merge(keys, w):
    u, inv = np.unique(keys, return_inverse=True)
    p = np.bincount(inv.reshape(-1), weights=w)
    keep = p > 0
    return u[keep], p[keep]


def _law(H, init_lab, init_act, variant=None, k=1):
    """Exact law of (labels, activities) after N_MCS MCS, as (keys, probs).
    k attempts per activation: 16 / k activations per MCS, colour alpha mod
    4, each making k attempts one after another in its sub-area (each sees
    the lattice and the counters the previous one left)."""
    R = LAM_ACT / MAX_ACT
    keys = _encode(init_lab.reshape(1, -1).astype(np.int64), init_act.reshape(1, -1).astype(np.int64))
    p = np.ones(1)
    for _ in range(N_MCS):
        for step in range(16):
            phi = (step // k) % 4
            cx, cy = phi & 1, (phi >> 1) & 1
            lab, act = _decode(keys)
            hk = H[(lab << np.arange(N)[None, :]).sum(axis=1)]
            gm = _gm(lab, act, variant)
            out_k, out_w = [keys], [p.copy()]
            for oy in range(2):
                for ox in range(2):
                    ty, tx = 2 * cy + oy, 2 * cx + ox
                    t = ty * L + tx
                    for dy, dx in _NB:
                        s = _site(ty + dy, tx + dx)
                        move = lab[:, t] != lab[:, s]
                        nl = lab.copy()
                        nl[:, t] = lab[:, s]
                        na = act.copy()
                        na[:, t] = np.where(lab[:, s] == 1, MAX_ACT, 0)
                        dh = H[(nl << np.arange(N)[None, :]).sum(axis=1)] - hk
                        if variant != "no_act":
                            sign = -1.0 if variant == "flipped" else 1.0
                            dh = dh + sign * R * (gm[:, t] - gm[:, s])
                        acc = np.where(dh <= 0, 1.0, np.exp(-np.maximum(dh, 0.0) / T))
                        f = np.where(move, acc, 0.0) * p / 32.0
                        out_k.append(_encode(nl, na))
                        out_w.append(f)
                        out_w[0] -= f
            keys, p = _merge(np.concatenate(out_k), np.concatenate(out_w))
        if variant != "no_decay":
            lab, act = _decode(keys)
            keys, p = _merge(_encode(lab, np.maximum(act - 1, 0)), p)
    return keys, p


def _chi2_pvalue(counts, expected):
    small = expected < 5
    obs = np.concatenate([counts[~small], [counts[small].sum()]])
    exp = np.concatenate([expected[~small], [expected[small].sum()]])
    keep = exp > 0
    obs, exp = obs[keep], exp[keep]
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    return stats.chi2.sf(chi2, len(obs) - 1)


def _initial():
    lab = np.zeros((L, L), dtype=np.int64)
    lab[1:3, 1:3] = 1
    act = np.zeros((L, L), dtype=np.int64)
    act[1:3, 1:3] = [[3, 1], [1, 3]]
    return lab, act


def _oracle_runs(k, seed):
    lab, act = _initial()
    m = oracle.Model(2, (L, L), [[0.0, J_CM], [J_CM, 0.0]], [0.0, LAM_V], [0, V_T], [0.0, LAM_S], [0, S_T],
                     lambda_act=[0.0, LAM_ACT], max_act=[0, MAX_ACT], T=T, s=2, k=k, seed=seed)
    fl, fa = oracle.replicates_act(m, lab, act, [0, 1], N_MCS, R_REP)
    # activities of medium sites are 0 by construction; the key holds them as they are
    return _encode(fl.astype(np.int64), fa.astype(np.int64))


@pytest.fixture(scope="module")
def runs():
    return _oracle_runs(1, 2024)


@pytest.fixture(scope="module")
def table():
    return _h_table()


def _counts(keys, law_keys):
    pos = np.searchsorted(law_keys, keys)
    pos = np.minimum(pos, len(law_keys) - 1)
    inside = law_keys[pos] == keys
    return np.bincount(pos[inside], minlength=len(law_keys)), int((~inside).sum())


def test_act_law_one_mcs(runs, table):
    lab, act = _initial()
    k, p = _law(table, lab, act)
    assert abs(p.sum() - 1.0) < 1e-9
    counts, outside = _counts(runs, k)
    # every sampled state is reachable under the law
    assert outside == 0
    assert _chi2_pvalue(counts, p * R_REP) > 1e-4
    # the law of the macrostate (volume, total activity)
    lk, ak = _decode(k)
    macro = lk.sum(axis=1) * 64 + ak.sum(axis=1)
    ls, as_ = _decode(runs)
    macro_s = ls.sum(axis=1) * 64 + as_.sum(axis=1)
    nb = int(max(macro.max(), macro_s.max())) + 1
    assert _chi2_pvalue(np.bincount(macro_s, minlength=nb), np.bincount(macro, weights=p, minlength=nb) * R_REP) > 1e-4


@pytest.mark.parametrize("variant", ["no_act", "flipped", "arithmetic", "all_neighbours", "no_decay"])
def test_act_law_has_power(runs, table, variant):
    lab, act = _initial()
    k, p = _law(table, lab, act, variant)
    counts, outside = _counts(runs, k)
    assert outside > 0 or _chi2_pvalue(counts, p * R_REP) < 1e-6


def test_act_law_four_attempts_per_activation(table):
    # k = 4: four activations per MCS, one per colour, each running its four
    # attempts back to back; the law of k = 1 (colours taking turns after
    # every attempt) is rejected by the same samples
    lab, act = _initial()
    keys = _oracle_runs(4, 77)
    k4, p4 = _law(table, lab, act, k=4)
    counts, outside = _counts(keys, k4)
    assert outside == 0
    assert _chi2_pvalue(counts, p4 * R_REP) > 1e-4
    k1, p1 = _law(table, lab, act, k=1)
    counts, outside = _counts(keys, k1)
    assert outside > 0 or _chi2_pvalue(counts, p1 * R_REP) < 1e-6
