"""Test-side definitions written straight from the paper's equations, for
pinning the oracle.  Independent of the oracle's C code.

Full Hamiltonian (Methods, eq. 1 + eq. 3) in 2^-16 fixed point:
  H = 1/2 sum_x sum_{n in Moore} J(tau(x), tau(x+n)) [sigma(x) != sigma(x+n)]
      + sum_{c >= 1} lambda_V(tau_c) (V(c) - V_t)^2 + lambda_S(tau_c) (S(c) - S_t)^2
with V(c) the number of sites of cell c and S(c) the number of (site of c,
Moore neighbour not of c) pairs.
"""
import itertools

import numpy as np


def q16(x):
    """Round-half-away-from-zero quantisation to 2^-16 units."""
    x = np.asarray(x, dtype=np.float64) * 65536.0
    return (np.sign(x) * np.floor(np.abs(x) + 0.5)).astype(np.int64)


def moore(ndim):
    rng = [(-1, 0, 1)] * ndim
    offs = [o for o in itertools.product(*rng) if any(o)]
    if ndim == 2:
        offs = [(0,) + o for o in offs]
    return offs  # tuples (dz, dy, dx)


def neighbour(lat, off):
    """nb[z,y,x] = lat[z+dz, y+dy, x+dx] with periodic wrap."""
    return np.roll(lat, shift=(-off[0], -off[1], -off[2]), axis=(0, 1, 2))


def site_types(lat, cell_type, obstacle_type):
    t = cell_type[np.maximum(lat, 0)]
    return np.where(lat < 0, obstacle_type, t)


def counts(lat, n_cells, ndim):
    lat = np.asarray(lat).reshape(lat.shape if lat.ndim == 3 else (1,) + lat.shape)
    V = np.bincount(lat[lat > 0].ravel(), minlength=n_cells + 1).astype(np.int64)
    S = np.zeros(n_cells + 1, dtype=np.int64)
    for off in moore(ndim):
        nb = neighbour(lat, off)
        m = (lat > 0) & (nb != lat)
        S += np.bincount(lat[m].ravel(), minlength=n_cells + 1)
    return V, S


def full_h(lat, cell_type, n_cells, ndim, J, lambda_V, V_target, lambda_S, S_target,
           obstacle_type=-1):
    lat = np.asarray(lat)
    Jq = q16(J)
    lv, ls = q16(lambda_V), q16(lambda_S)
    ct = np.asarray(cell_type)
    ty = site_types(lat, ct, obstacle_type)
    adh2 = 0
    for off in moore(ndim):
        nb = neighbour(lat, off)
        tn = neighbour(ty, off)
        adh2 += int(np.sum(Jq[ty, tn] * (lat != nb)))
    assert adh2 % 2 == 0
    V, S = counts(lat, n_cells, ndim)
    tc = ct[1:]
    vt = np.asarray(V_target)[tc]
    st = np.asarray(S_target)[tc]
    hv = int(np.sum(lv[tc] * (V[1:] - vt) ** 2))
    hs = int(np.sum(ls[tc] * (S[1:] - st) ** 2))
    return adh2 // 2 + hv + hs
