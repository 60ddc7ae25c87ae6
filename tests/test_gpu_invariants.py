"""Failure detection through the C ABI: cpm_check_invariants recounts volume
and surface on the device and compares them with the tracked counters (the
scheme's guarantee that a cell's tracked size equals its lattice count,
Results, "Designing a parallel execution scheme", Fig. 2B), and cpm_init /
cpm_batch_init reject lattices with labels out of range."""
import sys

import numpy as np
import pytest

from paper_2312_09317_amd import cpm, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cpm.load()
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _find_all(hay, needle):
    """Start indices of every occurrence of int32 sequence needle in hay."""
    n = needle.size
    win = np.lib.stride_tricks.sliding_window_view(hay, n)
    first = np.flatnonzero(hay[: hay.size - n + 1] == needle[0])
    return [int(i) for i in first if np.array_equal(win[i], needle)]


def test_clean_run_passes_and_corrupt_counter_fails(torch_cuda):
    torch = torch_cuda
    w = inputs.config0()
    _say("case config0: 10 MCS, then one counter corrupted in the workspace")
    sim = cpm.Simulation(cpm.Params.from_workload(w), w.lattice, w.cell_type)
    assert sim.check_invariants()
    sim.sweep(10)
    assert sim.check_invariants()
    v, s = sim.counters()
    torch.cuda.synchronize()
    # the exact (V, S) pairs of cells 1..n as the workspace holds them
    pairs = np.stack([v.cpu().numpy()[1:], s.cpu().numpy()[1:]], axis=1).reshape(-1).astype(np.int32)
    ws = sim.workspace.view(torch.int32).cpu().numpy().copy()
    hits = _find_all(ws, pairs)
    assert hits, "tracked counters not found in the workspace"
    bad = ws.copy()
    for h in hits:
        bad[h + 2 * 4] += 1  # volume of cell 5
    sim.workspace.view(torch.int32).copy_(torch.as_tensor(bad))
    assert not sim.check_invariants()
    # restored: the check itself changed nothing
    sim.workspace.view(torch.int32).copy_(torch.as_tensor(ws))
    assert sim.check_invariants()
    sim.sweep(2)
    assert sim.check_invariants()
    sim.close()


def test_lattice_written_behind_the_library(torch_cuda):
    torch = torch_cuda
    w = inputs.config0()
    _say("case config0: lattice sites rewritten after the sweep")
    sim = cpm.Simulation(cpm.Params.from_workload(w), w.lattice, w.cell_type)
    sim.sweep(3)
    flat = sim.lattice.view(-1)
    site = int(np.flatnonzero(sim.lattice.cpu().numpy().reshape(-1) == 3)[0])
    flat[site] = 4  # a valid label, but cell 3's and 4's counters are now stale
    assert not sim.check_invariants()
    flat[site] = 3
    assert sim.check_invariants()
    flat[site] = w.n_cells + 1  # out of range: caught before any recount
    assert not sim.check_invariants()
    flat[site] = -1  # obstacle in a model without an obstacle type
    assert not sim.check_invariants()
    flat[site] = 3
    assert sim.check_invariants()
    sim.close()


@pytest.mark.parametrize("bad", ["too_large", "below_minus_one", "obstacle_without_type"])
def test_init_rejects_labels_out_of_range(torch_cuda, bad):
    w = inputs.config0()
    lat = w.lattice.copy()
    lat.reshape(-1)[123] = {"too_large": w.n_cells + 1, "below_minus_one": -2, "obstacle_without_type": -1}[bad]
    _say(f"case init with a bad label: {bad}")
    with pytest.raises(cpm.CpmError) as e:
        cpm.Simulation(cpm.Params.from_workload(w), lat, w.cell_type)
    assert e.value.code == cpm.CPM_EINVAL


def test_batch_check_and_init(torch_cuda):
    torch = torch_cuda
    ws = inputs.config3(n_lattices=6, seed=3, L_min=24, L_max=40, n_mcs=4)
    _say("case batch of 6: check, then one lattice rewritten")
    b = cpm.Batch([cpm.Params.from_workload(w) for w in ws], [w.lattice for w in ws], [w.cell_type for w in ws])
    assert all(b.check_invariants())
    b.sweep(4)
    assert all(b.check_invariants())
    lat3 = b.lattice(3)
    i = int(np.flatnonzero(lat3.cpu().numpy().reshape(-1) >= 1)[0])
    old = int(lat3.reshape(-1)[i])
    lat3.reshape(-1)[i] = 0
    ok = b.check_invariants()
    assert ok == [True, True, True, False, True, True]
    lat3.reshape(-1)[i] = old
    assert all(b.check_invariants())
    b.close()
    lats = [w.lattice.copy() for w in ws]
    lats[2].reshape(-1)[0] = ws[2].n_cells + 1
    with pytest.raises(cpm.CpmError) as e:
        cpm.Batch([cpm.Params.from_workload(w) for w in ws], lats, [w.cell_type for w in ws])
    assert e.value.code == cpm.CPM_EINVAL
    torch.cuda.synchronize()
