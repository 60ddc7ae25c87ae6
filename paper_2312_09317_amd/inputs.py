"""Seeded synthetic inputs: initial lattices and parameter sets.

This module holds no arithmetic of the method itself: it only places cells
on a lattice and lists parameter values.  Both the GPU library's tests and the
oracle's tests draw their inputs from here, so the two sides see the same
initial states.  Random placement uses NumPy's PCG64 with the given seed.

Lattice convention: int32, shape (Lz, Ly, Lx) (x fastest in memory), values
-1 = obstacle, 0 = medium, 1..C = cells.  ``cell_type`` has C+1 entries;
entry 0 is the medium type 0.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Moore-26 interface count of the digitised ball x^2+y^2+z^2 <= 24 (485
# voxels), the ball whose volume is nearest to 500 (the r^2 <= 25 ball has
# 515 voxels; the tie is broken towards the smaller ball).  Checked by a test
# against the oracle's recount.
S_TARGET_BALL_V500 = 2690
# The same count for x^2+y^2+z^2 <= 38 (1021 voxels), the ball nearest to
# V = 1000.
S_TARGET_BALL_V1000 = 4490


@dataclass
class Workload:
    """A lattice, its cells' types and the model parameters for one run."""
    name: str
    ndim: int
    dims: tuple                 # (Lx, Ly, Lz); Lz = 1 in 2D
    lattice: np.ndarray         # int32, shape (Lz, Ly, Lx)
    cell_type: np.ndarray       # int32, C+1 entries
    J: np.ndarray               # float64, n_types x n_types
    lambda_V: np.ndarray
    V_target: np.ndarray
    lambda_S: np.ndarray
    S_target: np.ndarray
    T: float
    n_mcs: int
    seed: int = 1
    lattice_id: int = 0
    s: int = 2
    k: int = 1
    obstacle_type: int = -1
    lambda_act: Optional[np.ndarray] = None
    max_act: Optional[np.ndarray] = None
    act: Optional[np.ndarray] = None   # uint8, same shape as lattice
    lambda_P: Optional[np.ndarray] = None   # persistence strength per type (None: off)
    mu_P: Optional[np.ndarray] = None       # weight of the previous direction per type
    dt_P: int = 1                           # MCS looked back for the displacement
    lambda_C: Optional[np.ndarray] = None   # chemotaxis strength per type (None: off)
    C_field: Optional[np.ndarray] = None    # int16, ndim components per site, units of 2^-14
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return len(self.cell_type) - 1

    @property
    def n_sites(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


def _two_type(j_cc, j_cm, lam_v, v_t, lam_s=0.0, s_t=0):
    J = np.array([[0.0, j_cm], [j_cm, j_cc]])
    return (J, np.array([0.0, lam_v]), np.array([0, v_t], dtype=np.int32),
            np.array([0.0, lam_s]), np.array([0, s_t], dtype=np.int32))


def squares_2d(L=100, n_cells=20, side=10, seed=1):
    """n_cells squares of side `side` at seeded random non-overlapping
    positions on an L x L periodic lattice (squares may wrap around)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lat = np.zeros((L, L), dtype=np.int32)
    placed = 0
    tries = 0
    while placed < n_cells:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place squares")
        x0, y0 = rng.integers(0, L, size=2)
        ys = (y0 + np.arange(side)) % L
        xs = (x0 + np.arange(side)) % L
        if np.any(lat[np.ix_(ys, xs)] != 0):
            continue
        placed += 1
        lat[np.ix_(ys, xs)] = placed
    return lat.reshape(1, L, L)


def jittered_cubes(L=256, grid=27, edge=8, seed=1):
    """grid^3 cubes of edge `edge` on an L^3 periodic lattice: cell (i,j,k)
    sits in the box starting at floor(i*L/grid) (per axis), shifted by an
    integer jitter drawn uniformly from [0, w - edge] where w is the box
    width."""
    rng = np.random.Generator(np.random.PCG64(seed))
    starts = [(i * L) // grid for i in range(grid)] + [L]
    widths = np.diff(starts)
    if widths.min() < edge:
        raise ValueError("cubes do not fit their grid boxes")
    lat = np.zeros((L, L, L), dtype=np.int32)
    cid = 0
    for kz in range(grid):
        for jy in range(grid):
            for ix in range(grid):
                cid += 1
                jit = rng.integers(0, np.array([widths[ix], widths[jy], widths[kz]]) - edge + 1)
                x0 = starts[ix] + jit[0]
                y0 = starts[jy] + jit[1]
                z0 = starts[kz] + jit[2]
                lat[z0:z0 + edge, y0:y0 + edge, x0:x0 + edge] = cid
    return lat


def config0(seed=1):
    """2D, 100x100 periodic, 20 cells as 10x10 squares, J(cell,cell)=20,
    J(cell,medium)=10, lambda_V=50, V_target=100, T=20, 100 MCS."""
    lat = squares_2d(100, 20, 10, seed)
    J, lv, vt, ls, st = _two_type(20.0, 10.0, 50.0, 100)
    return Workload("2d-100x100-20cells", 2, (100, 100, 1), lat,
                    np.array([0] + [1] * 20, dtype=np.int32), J, lv, vt, ls, st,
                    T=20.0, n_mcs=100, seed=seed)


def config1(L=256, grid=27, seed=1, n_mcs=1000):
    """3D, L^3 periodic, grid^3 cubes of 8^3 on a jittered grid,
    J(cell,cell)=40, J(cell,medium)=20, lambda_V=25, V_target=500,
    lambda_S=0.5, S_target=2690, T=20.  L=256, grid=27 is the full-size
    workload (19,683 cells); smaller L / grid give the same structure for
    quick parity runs."""
    lat = jittered_cubes(L, grid, 8, seed)
    n = grid ** 3
    J, lv, vt, ls, st = _two_type(40.0, 20.0, 25.0, 500, 0.5, S_TARGET_BALL_V500)
    return Workload(f"3d-{L}^3-{n}cells", 3, (L, L, L), lat,
                    np.array([0] + [1] * n, dtype=np.int32), J, lv, vt, ls, st,
                    T=20.0, n_mcs=n_mcs, seed=seed)


def gaussian_field(L, corr=12.0, seed=1, workers=None):
    """Periodic Gaussian random field on an L^3 lattice (float32): seeded
    white noise convolved with a Gaussian kernel of standard deviation
    corr / sqrt(2), so that the field's covariance is a Gaussian of standard
    deviation `corr` voxels.  Done in Fourier space with scipy's float32
    FFT."""
    import os
    import scipy.fft
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((L, L, L), dtype=np.float32)
    w = workers or min(16, os.cpu_count() or 1)
    spec = scipy.fft.rfftn(noise, workers=w)
    del noise
    sk = corr / np.sqrt(2.0)
    k = np.fft.fftfreq(L).astype(np.float32)
    kr = np.fft.rfftfreq(L).astype(np.float32)
    c = np.float32(-2.0 * np.pi ** 2 * sk ** 2)
    gz = np.exp(c * k * k)[:, None, None]
    gy = np.exp(c * k * k)[None, :, None]
    gx = np.exp(c * kr * kr)[None, None, :]
    spec *= gz
    spec *= gy
    spec *= gx
    return scipy.fft.irfftn(spec, s=(L, L, L), workers=w).astype(np.float32, copy=False)


def config2(L=1024, grid=100, seed=1, n_mcs=200, edge=8, corr=12.0, obstacle_frac=0.3, min_voxels=64,
            motile_frac=0.5):
    """3D tissue-scale CPM: an L^3 periodic lattice whose static obstacle
    (label -1, type 3) is the top `obstacle_frac` of a Gaussian random field
    of correlation length `corr`; cells seeded as grid^3 jittered cubes of
    `edge` (as in config1), clipped to the free voxels, cells left with fewer
    than `min_voxels` voxels dropped and the rest relabelled 1..C in seeding
    order; each cell motile (type 1, Act term lambda_act 300, Max_act 30) or
    not (type 2) by a seeded draw with probability `motile_frac`.  Energies
    as config1 (J_cc 40, J_cm 20, lambda_V 25, lambda_S 0.5) with V_target
    1000 and S_target 4490; J(cell, obstacle) = J(cell, medium), J(medium,
    obstacle) = 0; T = 20.  L = 1024, grid = 100 is the full-size workload."""
    field = gaussian_field(L, corr, seed)
    flat = field.reshape(-1)
    cut = np.partition(flat, int((1.0 - obstacle_frac) * flat.size))[int((1.0 - obstacle_frac) * flat.size)]
    obstacle = field > cut
    del field, flat
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    starts = np.array([(i * L) // grid for i in range(grid)] + [L])
    widths = np.diff(starts)
    if widths.min() < edge:
        raise ValueError("cubes do not fit their grid boxes")
    iz, iy, ix = np.meshgrid(np.arange(grid), np.arange(grid), np.arange(grid), indexing="ij")
    iz, iy, ix = iz.reshape(-1), iy.reshape(-1), ix.reshape(-1)
    jit = rng.integers(0, np.stack([widths[ix], widths[iy], widths[iz]], axis=1) - edge + 1)
    x0, y0, z0 = starts[ix] + jit[:, 0], starts[iy] + jit[:, 1], starts[iz] + jit[:, 2]
    lat = np.zeros((L, L, L), dtype=np.int32)
    ids = np.arange(1, grid ** 3 + 1, dtype=np.int32)
    for dz in range(edge):
        for dy in range(edge):
            lat[(z0 + dz)[:, None], (y0 + dy)[:, None], x0[:, None] + np.arange(edge)[None, :]] = ids[:, None]
    lat[obstacle] = -1
    del obstacle
    vol = np.bincount(lat.reshape(-1)[lat.reshape(-1) > 0], minlength=grid ** 3 + 1)
    keep = vol >= min_voxels
    keep[0] = False
    remap = np.zeros(grid ** 3 + 2, dtype=np.int32)  # index 0 (medium) -> 0; -1 indexes the last entry
    remap[-1] = -1
    remap[np.nonzero(keep)[0]] = np.arange(1, int(keep.sum()) + 1, dtype=np.int32)
    lat = remap[lat]
    n = int(keep.sum())
    motile = rng.random(n) < motile_frac
    cell_type = np.concatenate([[0], np.where(motile, 1, 2)]).astype(np.int32)
    J = np.array([[0.0, 20.0, 20.0, 0.0], [20.0, 40.0, 40.0, 20.0], [20.0, 40.0, 40.0, 20.0], [0.0, 20.0, 20.0, 0.0]])
    w = Workload(f"3d-{L}^3-tissue-{n}cells", 3, (L, L, L), lat, cell_type, J,
                 np.array([0.0, 25.0, 25.0, 0.0]), np.array([0, 1000, 1000, 0], dtype=np.int32),
                 np.array([0.0, 0.5, 0.5, 0.0]), np.array([0, S_TARGET_BALL_V1000, S_TARGET_BALL_V1000, 0],
                                                          dtype=np.int32),
                 T=20.0, n_mcs=n_mcs, seed=seed, obstacle_type=3,
                 lambda_act=np.array([0.0, 300.0, 0.0, 0.0]), max_act=np.array([0, 30, 0, 0], dtype=np.int32),
                 act=np.zeros((L, L, L), dtype=np.uint8))
    w.extra["obstacle_voxels"] = int((lat < 0).sum())
    return w


def collective_3d(L=256, density=0.5, seed=1, n_mcs=200, lambda_p=40.0, mu=0.95, dt=15):
    """A packed 3D collective of persistently moving cells: cubes of edge 5
    on a jittered grid of an L^3 periodic lattice, as many as put cells of
    the target volume 150 at `density` of the lattice (grid^3 cells, grid =
    round((density L^3 / 150)^(1/3)); 38^3 = 54,872 at L = 256, density
    0.5).  The paper's 3D settings: V_target 150, lambda_V 25, surface
    target 1500, lambda_surface 0.2, J(cell, cell) 10, T 20; for the
    collective J(cell, medium) 0, mu 0.95, dt 15 MCS, lambda_persistence 40."""
    grid = max(1, int(round((density * L ** 3 / 150.0) ** (1.0 / 3.0))))
    lat = jittered_cubes(L, grid, 5, seed)
    n = grid ** 3
    J, lv, vt, ls, st = _two_type(10.0, 0.0, 25.0, 150, 0.2, 1500)
    w = Workload(f"3d-{L}^3-collective-{n}cells", 3, (L, L, L), lat,
                 np.array([0] + [1] * n, dtype=np.int32), J, lv, vt, ls, st,
                 T=20.0, n_mcs=n_mcs, seed=seed)
    w.lambda_P = np.array([0.0, lambda_p])
    w.mu_P = np.array([0.0, mu])
    w.dt_P = int(dt)
    w.extra["density"] = n * 150.0 / float(L) ** 3
    return w


def circular_field(L):
    """The paper's circular chemotaxis field on an L x L lattice: at every
    site the unit vector at 90 degrees (counter-clockwise) to the radial
    vector from the lattice centre to the site's centre, as int16 in units of
    2^-14 (x, y per site, sites in lattice order).  For odd L one site centre
    is the lattice centre, where the direction is undefined: its vector is
    zero."""
    c = L / 2.0
    y, x = np.mgrid[0:L, 0:L].astype(np.float64)
    rx, ry = x + 0.5 - c, y + 0.5 - c
    r = np.hypot(rx, ry)
    rr = np.where(r > 0, r, 1.0)
    f = np.where((r > 0)[..., None], np.stack([-ry / rr, rx / rr], axis=-1), 0.0)
    return np.rint(f * 16384.0).astype(np.int16).reshape(-1)


def chemotaxis_2d(L=256, n_cells=8, side=50, radius=None, seed=1, n_mcs=200, lambda_chem=10.0):
    """Cells circling in the circular chemotaxis field (Fig. 5A, Fig. 6A/E):
    n_cells squares of side `side` centred on a ring of radius `radius`
    (default 0.35 L) about the lattice centre at equal angles, the first at a
    seeded random angle.  The paper's 2D settings (V_target 2500, surface
    target 600, lambda_surface 2, J(cell, medium) 10, T 10) with lambda_V 20
    and lambda_chemotaxis 10; J(cell, cell) = 20 (not given)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radius = 0.35 * L if radius is None else radius
    lat = np.zeros((L, L), dtype=np.int32)
    phase = rng.random() * 2 * np.pi
    for i in range(n_cells):
        ang = phase + 2 * np.pi * i / n_cells
        cx = int(round(L / 2 + radius * np.cos(ang))) - side // 2
        cy = int(round(L / 2 + radius * np.sin(ang))) - side // 2
        ys = (cy + np.arange(side)) % L
        xs = (cx + np.arange(side)) % L
        if np.any(lat[np.ix_(ys, xs)] != 0):
            raise ValueError("cells overlap on the ring")
        lat[np.ix_(ys, xs)] = i + 1
    J, lv, vt, ls, st = _two_type(20.0, 10.0, 20.0, 2500, 2.0, 600)
    w = Workload(f"2d-{L}x{L}-chemotaxis-{n_cells}cells", 2, (L, L, 1), lat.reshape(1, L, L),
                 np.array([0] + [1] * n_cells, dtype=np.int32), J, lv, vt, ls, st,
                 T=10.0, n_mcs=n_mcs, seed=seed)
    w.lambda_C = np.array([0.0, lambda_chem])
    w.C_field = circular_field(L)
    return w


def act_2d(L=200, side=50, lambda_act=200.0, max_act=50, seed=1, n_mcs=750):
    """One cell, a side x side square in the middle of an L x L lattice, with
    the Act term (Fig. 5B, Fig. 6B): the paper's 2D settings (V_target 2500,
    surface target 600, lambda_surface 2, J(cell, medium) 10, T 10) with
    lambda_V 20, Max_act 50 and polarisation strength lambda_act."""
    lat = np.zeros((L, L), dtype=np.int32)
    o = (L - side) // 2
    lat[o:o + side, o:o + side] = 1
    J, lv, vt, ls, st = _two_type(0.0, 10.0, 20.0, 2500, 2.0, 600)
    w = Workload(f"2d-{L}x{L}-act-lambda{lambda_act:g}", 2, (L, L, 1), lat.reshape(1, L, L),
                 np.array([0, 1], dtype=np.int32), J, lv, vt, ls, st, T=10.0, n_mcs=n_mcs, seed=seed)
    w.lambda_act = np.array([0.0, float(lambda_act)])
    w.max_act = np.array([0, int(max_act)], dtype=np.int32)
    return w


def sorting_2d(L=2048, side=50, seed=1, n_mcs=1000, density=0.95, j_same=5.0, j_diff=15.0, j_medium=10.0):
    """Two-type cell sorting in 2D: side x side squares on a jittered grid
    filling about `density` of an L x L lattice (squares_jittered_2d; 40 x 40
    = 1,600 cells at L = 2048), each cell of type 1 or 2 by a seeded fair
    draw.  The paper's settings for all its 2D runs: V_target 2500, surface
    target 600, lambda_surface 2, J(cell, medium) 10, T 10; lambda_V 20;
    differential adhesion J(1,1) = J(2,2) = j_same < J(1,2) = j_diff (like
    types adhere more strongly, so the populations sort)."""
    lat, n = squares_jittered_2d(L, density, side, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    types = np.concatenate([[0], 1 + (rng.random(n) < 0.5)]).astype(np.int32)
    J = np.array([[0.0, j_medium, j_medium], [j_medium, j_same, j_diff], [j_medium, j_diff, j_same]])
    return Workload(f"2d-{L}x{L}-sorting-{n}cells", 2, (L, L, 1), lat, types, J,
                    np.array([0.0, 20.0, 20.0]), np.array([0, 2500, 2500], dtype=np.int32),
                    np.array([0.0, 2.0, 2.0]), np.array([0, 600, 600], dtype=np.int32),
                    T=10.0, n_mcs=n_mcs, seed=seed)


def random_labels(dims, n_labels, seed, p_obstacle=0.0):
    """Uniform random labels 0..n_labels-1 (and -1 with probability
    p_obstacle): a maximally rough state that exercises every branch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lx, Ly, Lz = dims
    lat = rng.integers(0, n_labels, size=(Lz, Ly, Lx)).astype(np.int32)
    if p_obstacle > 0:
        lat[rng.random(lat.shape) < p_obstacle] = -1
    return lat


def random_blobs(dims, n_cells, seed, fill=0.6, p_obstacle=0.0):
    """Cells grown as random boxes on a medium background: realistic
    interfaces at small sizes.  Boxes may overlap; later ones overwrite."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lx, Ly, Lz = dims
    lat = np.zeros((Lz, Ly, Lx), dtype=np.int32)
    n_sites = Lx * Ly * Lz
    per = max(1, int(fill * n_sites / max(n_cells, 1)))
    edge = max(1, int(round(per ** (1.0 / (3 if Lz > 1 else 2)))))
    for c in range(1, n_cells + 1):
        x0, y0, z0 = rng.integers(0, Lx), rng.integers(0, Ly), rng.integers(0, Lz)
        ex = rng.integers(max(1, edge - 1), edge + 2)
        ey = rng.integers(max(1, edge - 1), edge + 2)
        ez = rng.integers(max(1, edge - 1), edge + 2) if Lz > 1 else 1
        xs = (x0 + np.arange(ex)) % Lx
        ys = (y0 + np.arange(ey)) % Ly
        zs = (z0 + np.arange(ez)) % Lz
        lat[np.ix_(zs, ys, xs)] = c
    if p_obstacle > 0:
        lat[(lat == 0) & (rng.random(lat.shape) < p_obstacle)] = -1
    return lat


def squares_jittered_2d(L, density=0.3, side=10, seed=1):
    """Squares of `side` on a jittered grid of an L x L lattice, filling about
    `density` of it: n = round(L sqrt(density) / side) squares per axis, one in
    each grid box, with an integer jitter drawn from [0, box - side]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = max(1, int(round(L * np.sqrt(density) / side)))
    starts = [(i * L) // n for i in range(n)] + [L]
    widths = np.diff(starts)
    if widths.min() < side:
        raise ValueError("squares do not fit their grid boxes")
    lat = np.zeros((L, L), dtype=np.int32)
    cid = 0
    for j in range(n):
        for i in range(n):
            cid += 1
            jx = rng.integers(0, widths[i] - side + 1)
            jy = rng.integers(0, widths[j] - side + 1)
            y0, x0 = starts[j] + jy, starts[i] + jx
            lat[y0:y0 + side, x0:x0 + side] = cid
    return lat.reshape(1, L, L), cid


def config3_points(n_lattices=512, L_min=64, L_max=512, seed=1):
    """The per-lattice draws of config3, without building lattices: side L
    uniform over the multiples of 4 in [L_min, L_max], then lambda_V, J_cc,
    J_cm, T and lambda_act log-uniform within a factor 4 of 50, 20, 10, 20,
    300, one lattice after another from one PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = np.arange(L_min, L_max + 1, 4)
    out = []
    for _ in range(n_lattices):
        L = int(rng.choice(sides))
        f = np.exp(rng.uniform(np.log(0.25), np.log(4.0), size=5))
        out.append(dict(lambda_V=50.0 * f[0], J_cc=20.0 * f[1], J_cm=10.0 * f[2], T=20.0 * f[3],
                        lambda_act=300.0 * f[4], L=L))
    return out


def config3_workload(p, i, seed=1, n_mcs=500, max_act=30):
    """Lattice i of config3 from its draws p: cells seeded at 30% density as
    10x10 squares (V_target = 100), Max_act = 30, s = 2, k = 1,
    lattice_id = i."""
    L = p["L"]
    lat, n = squares_jittered_2d(L, 0.3, 10, seed=seed * 100003 + i)
    J, lv, vt, ls, st = _two_type(p["J_cc"], p["J_cm"], p["lambda_V"], 100)
    w = Workload(f"2d-{L}x{L}-batch{i}", 2, (L, L, 1), lat, np.array([0] + [1] * n, dtype=np.int32),
                 J, lv, vt, ls, st, T=float(p["T"]), n_mcs=n_mcs, seed=seed, lattice_id=i,
                 lambda_act=np.array([0.0, p["lambda_act"]]), max_act=np.array([0, max_act], dtype=np.int32))
    w.extra["params"] = dict(p)
    return w


def config3(n_lattices=512, L_min=64, L_max=512, seed=1, n_mcs=500, max_act=30):
    """Batched 2D CPM: n_lattices independent lattices with side lengths drawn
    uniformly from the multiples of 4 in [L_min, L_max], cells seeded at 30%
    density as 10x10 squares (V_target = 100), and per-lattice lambda_V, J_cc,
    J_cm, T and lambda_act drawn log-uniformly within a factor 4 of the 2D
    base values (lambda_V 50, J_cc 20, J_cm 10, T 20, lambda_act 300);
    Max_act = 30, s = 2, k = 1.  Lattice i has lattice_id i."""
    return [config3_workload(p, i, seed, n_mcs, max_act)
            for i, p in enumerate(config3_points(n_lattices, L_min, L_max, seed))]


def mlp_weights(seed=0, sizes=(6, 256, 256, 256, 8)):
    """Initial weights of a multilayer perceptron: W[l] (out x in) uniform in
    +-sqrt(6 / in) (He-style), b[l] zero, drawn from a seeded PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, b = [], []
    for i in range(len(sizes) - 1):
        bound = np.sqrt(6.0 / sizes[i])
        W.append(rng.uniform(-bound, bound, size=(sizes[i + 1], sizes[i])))
        b.append(np.zeros(sizes[i + 1]))
    return W, b
