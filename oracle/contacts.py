"""Contact statistics by cell type (test infrastructure only).

The read-out of the paper's cell sorting experiments (Results, cell sorting;
Fig. 4: the mixing is tracked through homotypic and heterotypic cell
borders).  Plain numpy: for every Moore offset, compare each site with its
periodic neighbour at that offset and count the ordered pairs (x, y) with
different labels, neither an obstacle, by (type of x, type of y); the medium
is type 0.
"""
import itertools

import numpy as np


def contact_matrix(lattice, cell_type, n_types, ndim):
    """lattice: int array (Lz, Ly, Lx) (Lz = 1 in 2D); cell_type: per label
    (entry 0 = medium).  Returns an n_types x n_types int64 matrix."""
    lat = np.asarray(lattice, dtype=np.int64)
    if lat.ndim == 2:
        lat = lat[None]
    types = np.asarray(cell_type, dtype=np.int64).copy()
    types[0] = 0
    t_here = np.where(lat > 0, types[np.maximum(lat, 0)], 0)
    out = np.zeros((n_types, n_types), dtype=np.int64)
    zs = (-1, 0, 1) if ndim == 3 else (0,)
    for dz, dy, dx in itertools.product(zs, (-1, 0, 1), (-1, 0, 1)):
        if dz == dy == dx == 0:
            continue
        nb = np.roll(lat, shift=(-dz, -dy, -dx), axis=(0, 1, 2))  # nb[x] = lat[x + offset]
        t_nb = np.where(nb > 0, types[np.maximum(nb, 0)], 0)
        mask = (lat != nb) & (lat >= 0) & (nb >= 0)
        np.add.at(out, (t_here[mask], t_nb[mask]), 1)
    return out


def homotypic_fraction(m):
    """Share of cell-cell contacts (both types >= 1) between cells of the same type."""
    m = np.asarray(m)
    cc = m[1:, 1:]
    tot = cc.sum()
    return float(np.trace(cc) / tot) if tot else float("nan")
