"""GPU checks of the speed/accuracy harness (Fig. 5A, Fig. 6E): the serial and
parallel ensembles' occupancy counts equal those of the oracle's runs of the
same lattice ids, and a small study reports sane accuracies."""
import numpy as np
import pytest

import oracle
from oracle import accuracy as ref_acc
from paper_2312_09317_amd import accuracy, inputs

from tests.test_gpu_parity import _say, oracle_model, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def _small():
    return inputs.chemotaxis_2d(L=64, n_cells=3, side=16, radius=18, n_mcs=6)


@pytest.mark.parametrize("mode,s,k", [("serial", None, None), ("parallel", 2, 1), ("parallel", 4, 8)])
def test_ensemble_counts_match_oracle(torch_cuda, mode, s, k):
    w = _small()
    n_runs, n_mcs = 5, 6
    _say(f"ensemble {mode} s={s} k={k}: {n_runs} runs x {n_mcs} MCS")
    counts, _, stats, _ = accuracy.run_ensemble(w, n_runs, n_mcs, mode, s=s, k=k, id0=10)
    lats = []
    for r in range(n_runs):
        w.lattice_id = 10 + r
        if s is not None:
            w.s, w.k = s, k
        st = oracle.State(oracle_model(w), w.lattice, w.cell_type)
        st.serial_sweep(n_mcs) if mode == "serial" else st.sweep(n_mcs)
        lats.append(st.lattice)
    np.testing.assert_array_equal(counts, np.sum(np.asarray(lats) > 0, axis=0))
    assert counts.max() <= n_runs and stats[2] > 0


def test_small_study(torch_cuda):
    w = _small()
    out = accuracy.study(w, [(2, 1), (8, 8)], n_runs=32, n_mcs=20)
    assert 0.0 < out["noise_floor_accuracy"] <= 1.0
    for row in out["parallel"]:
        assert row["accuracy"] <= 1.0 and row["attempts_per_s"] > 0
    # the scoring is the reference definition
    a = ref_acc.cross_entropy(np.full(4, 0.5), np.full(4, 0.5), 32).mean()
    assert np.isclose(a, 1.0)
