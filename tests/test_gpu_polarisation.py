"""GPU checks of the directional-autocorrelation read-out (Fig. 5B): per-lag
sums and pair counts of every lattice of a batch equal the reference's on the
same samples, and a small serial-vs-parallel study runs end to end."""
import numpy as np
import pytest

from oracle import summary as ref_summary
from paper_2312_09317_amd import cpm, inputs, polarisation

from tests.test_gpu_parity import _say, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("serial", [False, True])
def test_autocorrelation_matches_reference(torch_cuda, serial):
    ws = [inputs.act_2d(L=64, side=16, lambda_act=lam) for lam in (0.0, 300.0, 800.0)]
    ws += inputs.config3(n_lattices=3, L_min=48, L_max=64, seed=9, n_mcs=0)
    params = [cpm.Params.from_workload(w, lattice_id=i) for i, w in enumerate(ws)]
    b = cpm.Batch(params, [w.lattice for w in ws], [w.cell_type for w in ws], [w.act for w in ws])
    n_samples, interval = 7, 4
    _say(f"autocorrelation: {len(ws)} lattices, {n_samples} samples every {interval} MCS, serial={serial}")
    samples = b.run_with_samples(2, n_samples, interval, serial=serial)
    ac = b.autocorrelation(samples, n_samples).cpu().numpy()
    smp = samples.cpu().numpy()
    defined = []
    for i, w in enumerate(ws):
        lo, hi = int(b.label_off[i]), int(b.label_off[i + 1])
        rec = smp[lo * n_samples * 5:hi * n_samples * 5].reshape(n_samples, hi - lo, 5)
        sums, counts = ref_summary.autocorrelation(rec[:, :, 0], rec[:, :, 2:2 + w.ndim], w.dims)
        np.testing.assert_array_equal(ac[i, :, 1], counts)
        np.testing.assert_allclose(ac[i, :, 0], sums, rtol=1e-12, atol=1e-12)
        defined.append(int(counts[0]))
    _say(f"defined unit steps per lattice: {defined}")
    assert sum(defined) > 0


def test_small_study(torch_cuda):
    out = polarisation.study(lambdas=(0.0, 600.0), n_runs=4, n_mcs=60, interval=10,
                             modes=(("serial", None, None), ("parallel", 2, 1)))
    for m in out["modes"]:
        A = np.asarray(m["A"])
        assert A.shape == (2, 6) and np.allclose(A[:, 0], 1.0) and np.all(np.abs(A) <= 1.0 + 1e-12)
