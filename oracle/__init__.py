"""Python access to the serial CPU oracle (test infrastructure only).

The oracle is a plain C implementation of the cellular Potts model sweep
under the paper's checkerboard parallel scheme (see cpm_oracle.c for the
definitions it follows).  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does.
"""
import ctypes
import os

import numpy as np

from .build import ensure_built

_lib = None


def lib():
    """The oracle library: the built one, or the file CPM_ORACLE_LIB names
    (e.g. a sanitizer build made by oracle.build.build(sanitize=True))."""
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(os.environ.get("CPM_ORACLE_LIB") or ensure_built())
        _declare(_lib)
    return _lib


class OrcModel(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("L", ctypes.c_int32 * 3),
        ("s", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("n_types", ctypes.c_int32),
        ("obstacle_type", ctypes.c_int32),
        ("T", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("lattice_id", ctypes.c_uint32),
        ("act_enabled", ctypes.c_int32),
        ("J", ctypes.POINTER(ctypes.c_double)),
        ("lambda_V", ctypes.POINTER(ctypes.c_double)),
        ("V_target", ctypes.POINTER(ctypes.c_int32)),
        ("lambda_S", ctypes.POINTER(ctypes.c_double)),
        ("S_target", ctypes.POINTER(ctypes.c_int32)),
        ("lambda_act", ctypes.POINTER(ctypes.c_double)),
        ("max_act", ctypes.POINTER(ctypes.c_int32)),
        ("lambda_P", ctypes.POINTER(ctypes.c_double)),
        ("mu_P", ctypes.POINTER(ctypes.c_double)),
        ("dt_P", ctypes.c_int32),
        ("lambda_C", ctypes.POINTER(ctypes.c_double)),
        ("C_field", ctypes.POINTER(ctypes.c_int16)),
    ]


_P = ctypes.c_void_p


def _declare(l):
    l.oracle_philox.argtypes = [_P, _P, _P]
    l.oracle_tables.argtypes = [ctypes.c_double, _P, ctypes.c_int32, _P, _P, _P]
    l.oracle_threshold.argtypes = [ctypes.c_double, _P, ctypes.c_int64, _P]
    l.oracle_recount.argtypes = [ctypes.POINTER(OrcModel), _P, ctypes.c_int32, _P, _P]
    l.oracle_cell_stats.argtypes = [ctypes.POINTER(OrcModel), _P, ctypes.c_int32, _P, _P, _P]
    l.oracle_delta_h.argtypes = [ctypes.POINTER(OrcModel), _P, _P, ctypes.c_int32, _P, _P, _P,
                                 ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _P, _P]
    l.oracle_persist_init.argtypes = [ctypes.POINTER(OrcModel), _P, ctypes.c_int32, _P, _P, _P]
    l.oracle_persist_update.argtypes = [ctypes.POINTER(OrcModel), _P, _P, ctypes.c_int32, _P, _P, _P]
    l.oracle_sweep_p.argtypes = [ctypes.POINTER(OrcModel), _P, _P, ctypes.c_int32, _P, _P, _P,
                                 ctypes.c_uint64, ctypes.c_int32, _P, _P, _P, _P]
    l.oracle_gm_act.argtypes = [ctypes.POINTER(OrcModel), _P, _P, ctypes.c_int32, _P,
                                ctypes.c_int64, _P]
    l.oracle_sweep.argtypes = [ctypes.POINTER(OrcModel), _P, _P, ctypes.c_int32, _P, _P, _P,
                               ctypes.c_uint64, ctypes.c_int32, _P, _P]
    l.oracle_serial_sweep.argtypes = [ctypes.POINTER(OrcModel), _P, _P, ctypes.c_int32, _P, _P, _P,
                                      ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, _P, _P]
    l.oracle_replicates.argtypes = [ctypes.POINTER(OrcModel), _P, _P, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, _P]
    l.oracle_replicates_act.argtypes = [ctypes.POINTER(OrcModel), _P, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, _P, _P]
    for f in ("oracle_replicates", "oracle_replicates_act", "oracle_philox", "oracle_tables", "oracle_threshold", "oracle_recount",
              "oracle_cell_stats", "oracle_delta_h", "oracle_gm_act", "oracle_sweep",
              "oracle_serial_sweep", "oracle_persist_init", "oracle_sweep_p", "oracle_persist_update"):
        getattr(l, f).restype = ctypes.c_int


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


class Model:
    """Holds a model description and the numpy buffers the C struct points at.

    Fields follow the cellular Potts model of the paper: J (n_types x n_types),
    per-type lambda_V / V_target (eq. 1), lambda_S / S_target (eq. 3),
    lambda_act / max_act (eq. 7), temperature T (eq. 2), plus the parallel
    scheme's sub-area edge s and attempts per activation k.
    """

    def __init__(self, ndim, dims, J, lambda_V, V_target, lambda_S=None, S_target=None,
                 lambda_act=None, max_act=None, T=20.0, seed=1, lattice_id=0, s=2, k=1,
                 obstacle_type=-1, lambda_P=None, mu_P=None, dt_P=1, lambda_C=None, C_field=None):
        n = len(lambda_V)
        self.J = np.ascontiguousarray(np.asarray(J, dtype=np.float64).reshape(n, n))
        self.lambda_V = np.ascontiguousarray(lambda_V, dtype=np.float64)
        self.V_target = np.ascontiguousarray(V_target, dtype=np.int32)
        self.lambda_S = np.ascontiguousarray(np.zeros(n) if lambda_S is None else lambda_S, dtype=np.float64)
        self.S_target = np.ascontiguousarray(np.zeros(n) if S_target is None else S_target, dtype=np.int32)
        self.act_enabled = lambda_act is not None
        self.lambda_act = np.ascontiguousarray(np.zeros(n) if lambda_act is None else lambda_act, dtype=np.float64)
        self.max_act = np.ascontiguousarray(np.zeros(n) if max_act is None else max_act, dtype=np.int32)
        dims = list(dims) + [1] * (3 - len(dims))
        self.c = OrcModel()
        self.c.ndim = ndim
        self.c.L = (ctypes.c_int32 * 3)(*dims)
        self.c.s = s
        self.c.k = k
        self.c.n_types = n
        self.c.obstacle_type = obstacle_type
        self.c.T = T
        self.c.seed = seed
        self.c.lattice_id = lattice_id
        self.c.act_enabled = 1 if self.act_enabled else 0
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        self.c.J = self.J.ctypes.data_as(dp)
        self.c.lambda_V = self.lambda_V.ctypes.data_as(dp)
        self.c.V_target = self.V_target.ctypes.data_as(ip)
        self.c.lambda_S = self.lambda_S.ctypes.data_as(dp)
        self.c.S_target = self.S_target.ctypes.data_as(ip)
        self.c.lambda_act = self.lambda_act.ctypes.data_as(dp)
        self.c.max_act = self.max_act.ctypes.data_as(ip)
        self.persistence = lambda_P is not None
        self.lambda_P = np.ascontiguousarray(np.zeros(n) if lambda_P is None else lambda_P, dtype=np.float64)
        self.mu_P = np.ascontiguousarray(np.zeros(n) if mu_P is None else mu_P, dtype=np.float64)
        self.c.lambda_P = self.lambda_P.ctypes.data_as(dp) if self.persistence else None
        self.c.mu_P = self.mu_P.ctypes.data_as(dp) if self.persistence else None
        self.c.dt_P = int(dt_P)
        # chemotaxis (eq. 4): per-type strength and the field C, int16 in
        # units of 2^-14, ndim components per site in lattice order
        self.chemotaxis = lambda_C is not None
        self.lambda_C = np.ascontiguousarray(np.zeros(n) if lambda_C is None else lambda_C, dtype=np.float64)
        self.C_field = None if C_field is None else np.ascontiguousarray(C_field, dtype=np.int16).reshape(-1)
        self.c.lambda_C = self.lambda_C.ctypes.data_as(dp) if self.chemotaxis else None
        self.c.C_field = self.C_field.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)) \
            if self.C_field is not None else None

    @property
    def dims(self):
        return tuple(self.c.L)

    @property
    def n_sites(self):
        L = self.c.L
        return L[0] * L[1] * L[2]


def philox(ctr, key):
    """Philox4x32-10 of one 128-bit counter (4 x u32) under a 64-bit key (2 x u32)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _check(lib().oracle_philox(_ptr(c), _ptr(k), _ptr(out)), "philox")
    return out


def tables(T):
    TI = np.zeros(8192, dtype=np.uint64)
    n = ctypes.c_int32(0)
    TM = np.zeros(256, dtype=np.uint64)
    TL = np.zeros(256, dtype=np.uint64)
    _check(lib().oracle_tables(T, _ptr(TI), 8192, ctypes.byref(n), _ptr(TM), _ptr(TL)), "tables")
    return TI[: n.value].copy(), TM, TL


def threshold(T, dh):
    dh = np.ascontiguousarray(dh, dtype=np.int64)
    out = np.zeros(dh.shape, dtype=np.uint64)
    _check(lib().oracle_threshold(T, _ptr(dh), dh.size, _ptr(out)), "threshold")
    return out


def recount(model, lattice, n_cells):
    lat = np.ascontiguousarray(lattice, dtype=np.int32)
    V = np.zeros(n_cells + 1, dtype=np.int64)
    S = np.zeros(n_cells + 1, dtype=np.int64)
    _check(lib().oracle_recount(ctypes.byref(model.c), _ptr(lat), n_cells, _ptr(V), _ptr(S)), "recount")
    return V, S


def cell_stats(model, lattice, n_cells):
    lat = np.ascontiguousarray(lattice, dtype=np.int32)
    V = np.zeros(n_cells + 1, dtype=np.int64)
    S = np.zeros(n_cells + 1, dtype=np.int64)
    cs = np.zeros((n_cells + 1, model.c.ndim), dtype=np.int64)
    _check(lib().oracle_cell_stats(ctypes.byref(model.c), _ptr(lat), n_cells, _ptr(V), _ptr(S), _ptr(cs)),
           "cell_stats")
    return V, S, cs


def delta_h(model, lattice, cell_type, V, S, t, src, new_label, act=None, P=None):
    lat = np.ascontiguousarray(lattice, dtype=np.int32)
    ct = np.ascontiguousarray(cell_type, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.int64)
    S = np.ascontiguousarray(S, dtype=np.int64)
    a = None if act is None else np.ascontiguousarray(act, dtype=np.uint8)
    p = None if P is None else np.ascontiguousarray(P, dtype=np.int32)
    out = ctypes.c_int64(0)
    _check(lib().oracle_delta_h(ctypes.byref(model.c), _ptr(lat), _ptr(ct), len(ct) - 1, _ptr(a),
                                _ptr(V), _ptr(S), int(t), int(src), int(new_label), ctypes.byref(out),
                                _ptr(p)), "delta_h")
    return out.value


def gm_act(model, lattice, cell_type, act, site):
    lat = np.ascontiguousarray(lattice, dtype=np.int32)
    ct = np.ascontiguousarray(cell_type, dtype=np.int32)
    a = np.ascontiguousarray(act, dtype=np.uint8)
    out = ctypes.c_int64(0)
    _check(lib().oracle_gm_act(ctypes.byref(model.c), _ptr(lat), _ptr(ct), len(ct) - 1, _ptr(a),
                               int(site), ctypes.byref(out)), "gm_act")
    return out.value


class State:
    """Lattice + per-cell counters advanced by the oracle in place."""

    def __init__(self, model, lattice, cell_type, act=None):
        self.model = model
        self.lattice = np.ascontiguousarray(lattice, dtype=np.int32).reshape(-1).copy()
        self.cell_type = np.ascontiguousarray(cell_type, dtype=np.int32)
        self.n_cells = len(self.cell_type) - 1
        if model.act_enabled:
            self.act = (np.zeros(self.lattice.size, dtype=np.uint8) if act is None
                        else np.ascontiguousarray(act, dtype=np.uint8).reshape(-1).copy())
        else:
            self.act = None
        self.V, self.S = recount(model, self.lattice, self.n_cells)
        self.mcs = 0
        self.stats = np.zeros(3, dtype=np.int64)
        self.P = self.hist = None
        if model.persistence:
            # per cell: direction (3 x 2^-14) and dt+1 centroids (3 x 2^-16)
            self.P = np.zeros((self.n_cells + 1) * 3, dtype=np.int32)
            self.hist = np.zeros((self.n_cells + 1) * (model.c.dt_P + 1) * 3, dtype=np.int64)
            self.p_t = np.zeros(1, dtype=np.int64)
            _check(lib().oracle_persist_init(ctypes.byref(model.c), _ptr(self.lattice), self.n_cells,
                                             _ptr(self.P), _ptr(self.hist), _ptr(self.p_t)), "persist_init")

    def sweep(self, n_mcs, target_log=None):
        if self.model.persistence:
            if target_log is not None:
                raise ValueError("target logs are not kept with persistence")
            rc = lib().oracle_sweep_p(ctypes.byref(self.model.c), _ptr(self.lattice), _ptr(self.cell_type),
                                      self.n_cells, _ptr(self.act), _ptr(self.V), _ptr(self.S),
                                      self.mcs, n_mcs, _ptr(self.stats), _ptr(self.P), _ptr(self.hist),
                                      _ptr(self.p_t))
        else:
            rc = lib().oracle_sweep(ctypes.byref(self.model.c), _ptr(self.lattice), _ptr(self.cell_type),
                                    self.n_cells, _ptr(self.act), _ptr(self.V), _ptr(self.S),
                                    self.mcs, n_mcs, _ptr(self.stats), _ptr(target_log))
        _check(rc, "sweep")
        self.mcs += n_mcs

    def serial_sweep(self, n_mcs, symmetric=False, target_log=None):
        rc = lib().oracle_serial_sweep(ctypes.byref(self.model.c), _ptr(self.lattice), _ptr(self.cell_type),
                                       self.n_cells, _ptr(self.act), _ptr(self.V), _ptr(self.S),
                                       self.mcs, n_mcs, 1 if symmetric else 0, _ptr(self.stats),
                                       _ptr(target_log))
        _check(rc, "serial_sweep")
        self.mcs += n_mcs


def replicates(model, lattice, cell_type, n_mcs, n_rep, mode="dcs"):
    """Final lattices of n_rep independent runs (replicate r uses lattice id
    model.lattice_id + r).  mode: "dcs" (parallel scheme), "serial",
    "symmetric" (serial, symmetric label proposal)."""
    lat = np.ascontiguousarray(lattice, dtype=np.int32).reshape(-1)
    ct = np.ascontiguousarray(cell_type, dtype=np.int32)
    out = np.zeros((n_rep, lat.size), dtype=np.int32)
    code = {"dcs": 0, "serial": 1, "symmetric": 2}[mode]
    _check(lib().oracle_replicates(ctypes.byref(model.c), _ptr(lat), _ptr(ct), len(ct) - 1, n_mcs,
                                   n_rep, code, _ptr(out)), "replicates")
    return out


def replicates_act(model, lattice, act, cell_type, n_mcs, n_rep):
    """Final lattices and activities of n_rep independent runs of an Act
    model under the parallel scheme, all starting from (lattice, act);
    replicate r uses lattice id model.lattice_id + r."""
    lat = np.ascontiguousarray(lattice, dtype=np.int32).reshape(-1)
    a0 = np.ascontiguousarray(act, dtype=np.uint8).reshape(-1)
    ct = np.ascontiguousarray(cell_type, dtype=np.int32)
    out_l = np.zeros((n_rep, lat.size), dtype=np.int32)
    out_a = np.zeros((n_rep, lat.size), dtype=np.uint8)
    _check(lib().oracle_replicates_act(ctypes.byref(model.c), _ptr(lat), _ptr(a0), _ptr(ct), len(ct) - 1,
                                       n_mcs, n_rep, _ptr(out_l), _ptr(out_a)), "replicates_act")
    return out_l, out_a


class Persistence:
    """Direction state of the persistence term for one lattice (eq. 5-6)."""

    def __init__(self, model, lattice, n_cells):
        self.model = model
        self.n_cells = n_cells
        self.P = np.zeros((n_cells + 1) * 3, dtype=np.int32)
        self.hist = np.zeros((n_cells + 1) * (model.c.dt_P + 1) * 3, dtype=np.int64)
        self.t = np.zeros(1, dtype=np.int64)
        lat = np.ascontiguousarray(lattice, dtype=np.int32).reshape(-1)
        _check(lib().oracle_persist_init(ctypes.byref(model.c), _ptr(lat), n_cells, _ptr(self.P),
                                         _ptr(self.hist), _ptr(self.t)), "persist_init")

    def update(self, lattice, cell_type):
        lat = np.ascontiguousarray(lattice, dtype=np.int32).reshape(-1)
        ct = np.ascontiguousarray(cell_type, dtype=np.int32)
        _check(lib().oracle_persist_update(ctypes.byref(self.model.c), _ptr(lat), _ptr(ct), self.n_cells,
                                           _ptr(self.P), _ptr(self.hist), _ptr(self.t)), "persist_update")
        return self.P.reshape(-1, 3)
