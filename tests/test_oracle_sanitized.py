"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs
sweeps of every model variant (adhesion, volume, surface, obstacles, the Act,
persistence and chemotaxis terms, several attempts per activation, the
serial CPM, 2D and 3D) without a report: no out-of-bounds access, no signed
overflow, no invalid shift in the checker the GPU library is held to."""
import os
import subprocess
import sys

import pytest

from oracle import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import ctypes
import sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle
# the sanitizer runtimes are live in this process, and the oracle is the instrumented build
ctypes.CDLL(None).__asan_report_load4
oracle.lib().__ubsan_handle_add_overflow
from paper_2312_09317_amd import inputs

def model(w, **over):
    kw = dict(lambda_act=w.lambda_act, max_act=w.max_act, T=w.T, seed=w.seed, lattice_id=w.lattice_id,
              s=w.s, k=w.k, obstacle_type=w.obstacle_type, lambda_P=w.lambda_P, mu_P=w.mu_P, dt_P=w.dt_P,
              lambda_C=w.lambda_C, C_field=w.C_field)
    kw.update(over)
    return oracle.Model(w.ndim, w.dims[:w.ndim], w.J, w.lambda_V, w.V_target, w.lambda_S, w.S_target, **kw)

w = inputs.config0()
st = oracle.State(model(w), w.lattice, w.cell_type); st.sweep(3); st.serial_sweep(1)
w = inputs.config1(L=24, grid=3, n_mcs=2)
st = oracle.State(model(w, k=8), w.lattice, w.cell_type); st.sweep(1)
w = inputs.config2(L=32, grid=3, n_mcs=2)
st = oracle.State(model(w), w.lattice, w.cell_type, w.act); st.sweep(2); st.serial_sweep(1)
w = inputs.collective_3d(L=24, n_mcs=2)
st = oracle.State(model(w), w.lattice, w.cell_type); st.sweep(2)
w = inputs.chemotaxis_2d(L=48, n_cells=2, side=12, radius=14, n_mcs=2)
st = oracle.State(model(w, s=4, k=16), w.lattice, w.cell_type); st.sweep(2); st.serial_sweep(1)
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    lib = build.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc's libasan is not installed")
    env = dict(os.environ, CPM_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:exitcode=24:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", f"ROOT = {ROOT!r}\n" + SCRIPT], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
