"""Cell-level summary statistics of a CPM run (test infrastructure only).

Plain numpy, float64.  The statistics are of the kinds the paper uses to
characterise motility (cell speed and directional persistence, Results,
"Emergent cell and tissue behavior is maintained", Fig. 5B; and the "Building
an image-based model" sections) plus volume and surface moments; the paper
gives no formula for them, so the definitions below are this project's
reading:

samples k = 0..K-1 taken every `interval` MCS; per cell c alive (V > 0) at a
sample, its centroid is centroid_sum / V reduced into [0, L) per axis.

* volume, surface: mean and population variance over all (cell, sample)
  pairs with the cell alive;
* speed: |d_k(c)| / interval over all pairs of consecutive samples with the
  cell alive at both, where d_k is the minimum-image centroid displacement;
* persistence: per cell, the directional autocorrelation
  A(tau) = mean_k u_k . u_{k+tau} of the unit displacement vectors (pairs
  where both are defined), A(0) = 1; the persistence time is the first lag at
  which A drops below 1/e, linearly interpolated between the two lags, in
  MCS; a cell whose A stays above 1/e gets the longest lag it has; mean and
  population variance over cells with at least one defined lag.

Output order: mean V, var V, mean S, var S, mean speed, var speed,
mean persistence, var persistence.
"""
import numpy as np

INV_E = float(np.exp(-1.0))


def centroids(vol, csum, dims):
    """vol: (C+1,), csum: (C+1, ndim) integer sums -> positions in [0, L)."""
    vol = np.asarray(vol, dtype=np.float64)
    csum = np.asarray(csum, dtype=np.float64)
    ndim = csum.shape[1]
    pos = np.zeros_like(csum)
    alive = vol > 0
    for d in range(ndim):
        x = np.zeros(len(vol))
        x[alive] = csum[alive, d] / vol[alive]
        x = np.fmod(x, dims[d])
        x[x < 0] += dims[d]
        pos[:, d] = x
    return pos


def summary(V, S, pos, dims, interval):
    """V, S: (K, C+1); pos: (K, C+1, ndim) centroid positions.  Entry 0 (the
    medium) is ignored."""
    V = np.asarray(V, dtype=np.float64)[:, 1:]
    S = np.asarray(S, dtype=np.float64)[:, 1:]
    pos = np.asarray(pos, dtype=np.float64)[:, 1:, :]
    K, C = V.shape
    L = np.asarray(dims[:pos.shape[2]], dtype=np.float64)
    alive = V > 0
    out = np.zeros(8)
    if alive.any():
        out[0], out[1] = V[alive].mean(), V[alive].var()
        out[2], out[3] = S[alive].mean(), S[alive].var()
    speeds = []
    persist = []
    for c in range(C):
        units = []
        for k in range(K - 1):
            if alive[k, c] and alive[k + 1, c]:
                d = pos[k + 1, c] - pos[k, c]
                d = d - L * np.rint(d / L)
                n = np.sqrt(np.sum(d * d))
                speeds.append(n / interval)
                units.append(d / n if n > 0 else None)
            else:
                units.append(None)
        m = len(units)
        # A(0) = 1; the crossing of 1/e is interpolated linearly between the
        # last lag where A was defined and the first where it falls below
        a_prev, last = 1.0, 0
        p = None
        any_lag = False
        for tau in range(1, m):
            vals = [float(np.dot(units[k], units[k + tau])) for k in range(m - tau)
                    if units[k] is not None and units[k + tau] is not None]
            if not vals:
                continue
            any_lag = True
            a = sum(vals) / len(vals)
            if a < INV_E:
                p = last + (tau - last) * (a_prev - INV_E) / (a_prev - a)
                break
            a_prev = a
            last = tau
        if not any_lag:
            continue
        if p is None:
            p = float(last)
        persist.append(p * interval)
    if speeds:
        sp = np.asarray(speeds)
        out[4], out[5] = sp.mean(), sp.var()
    if persist:
        pe = np.asarray(persist)
        out[6], out[7] = pe.mean(), pe.var()
    return out


def autocorrelation(V, pos, dims):
    """Directional autocorrelation of the cells of one run (Fig. 5B): for
    every lag tau = 0..K-2 (in sample intervals), the sum over cells c and
    steps k of u_k(c) . u_{k+tau}(c), the unit minimum-image displacements
    between consecutive samples (both defined: cell alive at the three or
    four samples involved and moved), and the number of such pairs.  Entry 0
    (the medium) is ignored.  Returns (sums, counts), each of length K - 1;
    their ratio is A(tau), and runs pool by adding sums and counts."""
    V = np.asarray(V, dtype=np.float64)[:, 1:]
    pos = np.asarray(pos, dtype=np.float64)[:, 1:, :]
    K, C = V.shape
    L = np.asarray(dims[:pos.shape[2]], dtype=np.float64)
    sums = np.zeros(K - 1)
    counts = np.zeros(K - 1)
    for c in range(C):
        units = []
        for k in range(K - 1):
            u = None
            if V[k, c] > 0 and V[k + 1, c] > 0:
                d = pos[k + 1, c] - pos[k, c]
                d = d - L * np.rint(d / L)
                n = np.sqrt(np.sum(d * d))
                if n > 0:
                    u = d / n
            units.append(u)
        for tau in range(K - 1):
            for k in range(K - 1 - tau):
                if units[k] is not None and units[k + tau] is not None:
                    sums[tau] += float(np.dot(units[k], units[k + tau]))
                    counts[tau] += 1
    return sums, counts
