"""The seeded workload generators against the model settings the paper prints
(Tables 1 and 2; fixture tests/golden/model_settings.json).  Parameters the
tables leave open (J between cells in 2D, the sorting energies) are the
generators' own and are not checked here."""
import json
import os

import numpy as np
import pytest

from paper_2312_09317_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "model_settings.json")


@pytest.fixture(scope="module")
def tables():
    with open(GOLDEN) as f:
        return json.load(f)


def _check_common_2d(w, c):
    assert w.V_target[1] == c["V_target"]
    assert w.S_target[1] == c["A_target"]
    assert w.lambda_S[1] == c["lambda_perimeter"]
    assert w.J[0, 1] == w.J[1, 0] == c["J_cell_ECM"]
    assert w.T == c["T"]


def test_chemotaxis_settings(tables):
    t = tables["table_1_2d"]
    w = inputs.chemotaxis_2d(L=128, n_cells=4, side=20)
    _check_common_2d(w, t["all_2d"])
    assert w.lambda_V[1] == t["chemotaxis"]["lambda_volume"]
    assert w.lambda_C[1] == t["chemotaxis"]["lambda_chemotaxis"]


def test_act_settings(tables):
    t = tables["table_1_2d"]
    r = t["act_polarisation"]
    w = inputs.act_2d()
    _check_common_2d(w, t["all_2d"])
    assert w.lambda_V[1] == r["lambda_volume"]
    assert w.max_act[1] == r["Max_act"]
    grid = np.arange(r["lambda_act_min"], r["lambda_act_max"] + 1, r["lambda_act_step"])
    assert w.lambda_act[1] in grid
    # the polarisation study's strengths: a zero control plus values on the paper's grid
    from paper_2312_09317_amd import polarisation
    import inspect
    lam = inspect.signature(polarisation.study).parameters["lambdas"].default
    assert all(x == 0 or x in grid for x in lam)


def test_sorting_uses_the_2d_settings(tables):
    w = inputs.sorting_2d(L=256)
    _check_common_2d(w, tables["table_1_2d"]["all_2d"])
    assert w.J[0, 2] == tables["table_1_2d"]["all_2d"]["J_cell_ECM"]


def test_collective_settings(tables):
    t = tables["table_2_3d"]
    c, r = t["all_3d"], t["collective"]
    w = inputs.collective_3d(L=64)
    assert w.V_target[1] == c["V_target"]
    assert w.lambda_V[1] == c["lambda_volume"]
    assert w.S_target[1] == c["A_target"]
    assert w.lambda_S[1] == c["lambda_perimeter"]
    assert w.J[1, 1] == c["J_cell_cell"]
    assert w.T == c["T"]
    assert w.mu_P[1] == r["mu"]
    assert w.dt_P == r["delta_t"]
    assert w.lambda_P[1] == r["lambda_persistence"]
    assert w.J[0, 1] == r["J_cell_ECM"]


@pytest.mark.parametrize("L", [64, 255, 256])
def test_circular_field(tables, L):
    f = tables["table_1_2d"]["chemotaxis_field"]
    v = inputs.circular_field(L).reshape(L, L, 2).astype(np.float64) / 16384.0
    y, x = np.mgrid[0:L, 0:L].astype(np.float64)
    rx, ry = x + 0.5 - L / 2.0, y + 0.5 - L / 2.0
    r = np.hypot(rx, ry)
    off = r > 0
    # unit length, within the 2^-14 rounding of each component
    assert np.abs(np.hypot(v[..., 0], v[..., 1])[off] - f["norm"]).max() < 2 ** -13
    # perpendicular to the radial vector, and counter-clockwise
    cos = (v[..., 0] * rx + v[..., 1] * ry)[off] / r[off]
    assert np.abs(cos).max() < 2 ** -13
    assert np.all((rx * v[..., 1] - ry * v[..., 0])[off] > 0)
    # the centre site of an odd lattice has no direction
    assert np.all(v[~off] == 0) and (~off).sum() == L % 2
    assert f["angle_to_radial_deg"] == 90
