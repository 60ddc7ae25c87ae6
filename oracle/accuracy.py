"""Ensemble agreement by pixel (cross-)entropy (Results, motility models;
Fig. 5A and Fig. 6E).  TEST INFRASTRUCTURE ONLY: only tests, the smoke check
and the benchmark's CPU-baseline leg may use this module.

Plain numpy, float64, written from the definitions:

* occupancy p(x): the fraction of an ensemble's runs whose final lattice holds
  a cell (label >= 1) at pixel x;
* binary entropy per pixel, in bits: H(p) = -p log2 p - (1 - p) log2(1 - p);
* cross-entropy of the parallel ensemble relative to the serial reference
  (reading: the reference is the distribution, the parallel ensemble the
  model): CE(x) = -p_ref log2 q - (1 - p_ref) log2(1 - q), where q is the
  parallel occupancy clipped to [1 / (2 n_par), 1 - 1 / (2 n_par)] (a pixel
  no parallel run occupied counts as half a run), averaged over all pixels;
* accuracy = 1 - mean CE (Fig. 6E).
"""
import numpy as np


def occupancy(lattices):
    """Fraction of runs (rows) holding a cell at each pixel (column)."""
    lat = np.asarray(lattices)
    return (lat.reshape(lat.shape[0], -1) >= 1).mean(axis=0)


def _xlog2(a, b):
    # a * log2(b) with 0 * log2(0) = 0
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.zeros(np.broadcast(a, b).shape)
    nz = a != 0
    out[nz] = (a * np.log2(np.where(b > 0, b, 1.0)))[nz]
    return out


def entropy(p):
    """Binary entropy of each pixel's occupancy, bits."""
    p = np.asarray(p, dtype=np.float64)
    return -(_xlog2(p, p) + _xlog2(1.0 - p, 1.0 - p))


def cross_entropy(p_ref, q_par, n_par):
    """Per-pixel cross-entropy (bits) of reference occupancy p_ref against
    the parallel occupancy q_par from n_par runs, clipped as above."""
    eps = 1.0 / (2.0 * n_par)
    q = np.clip(np.asarray(q_par, dtype=np.float64), eps, 1.0 - eps)
    p = np.asarray(p_ref, dtype=np.float64)
    return -(p * np.log2(q) + (1.0 - p) * np.log2(1.0 - q))


def accuracy(ref_lattices, par_lattices):
    """1 - mean pixel cross-entropy of a parallel ensemble against a serial one."""
    par = np.asarray(par_lattices)
    return 1.0 - float(cross_entropy(occupancy(ref_lattices), occupancy(par), par.shape[0]).mean())
