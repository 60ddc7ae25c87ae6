"""Directional persistence of Act-model cells under the serial CPM and the
parallel scheme (Results, motility models; Fig. 5B).

For each polarisation strength lambda_act, an ensemble of single-cell runs
(inputs.act_2d) is advanced as one batch, with the serial CPM or with the
parallel scheme at (s, k), and sampled every `interval` MCS; the library
reduces the samples to the directional autocorrelation of the cells' unit
displacements per lag (cpm_batch_autocorrelation), pooled here over the
ensemble.  The paper's finding is that persistence grows with lambda_act
under the serial CPM, and that a parallel scheme preserves it only when it
preserves the update statistics (k = 1 here; k = s^d runs each thread's
attempts back to back).
"""
import numpy as np

from . import cpm, inputs


def autocorrelation_curves(lambdas, n_runs, n_mcs, interval, mode="serial", s=2, k=1, id0=0, L=200,
                           device="cuda"):
    """A(tau) for tau = 0..n_mcs/interval - 1 per lambda (array, rows in
    lambdas order), mean speed per lambda, and the GPU milliseconds of the
    sweeps and reductions."""
    import torch
    ws, params = [], []
    for li, lam in enumerate(lambdas):
        for r in range(n_runs):
            w = inputs.act_2d(L=L, lambda_act=lam)
            ws.append(w)
            params.append(cpm.Params.from_workload(w, sub=s, attempts=k, lattice_id=id0 + li * n_runs + r))
    b = cpm.Batch(params, [w.lattice for w in ws], [w.cell_type for w in ws], [w.act for w in ws], device=device)
    n_samples = n_mcs // interval + 1
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    samples = b.run_with_samples(0, n_samples, interval, serial=(mode == "serial"))
    ac = b.autocorrelation(samples, n_samples)
    summ = b.summary(samples, n_samples, float(interval))
    e1.record()
    torch.cuda.synchronize()
    ac = ac.cpu().numpy().reshape(len(lambdas), n_runs, n_samples - 1, 2).sum(axis=1)
    curves = ac[..., 0] / np.maximum(ac[..., 1], 1.0)
    speed = summ.cpu().numpy()[:, 4].reshape(len(lambdas), n_runs).mean(axis=1)
    ms = e0.elapsed_time(e1)
    b.close()
    return curves, speed, ms


def study(lambdas=(0.0, 100.0, 200.0, 400.0, 800.0), n_runs=50, n_mcs=750, interval=50,
          modes=(("serial", None, None), ("parallel", 2, 1), ("parallel", 2, 4)), device="cuda", log=None):
    say = log or (lambda m: None)
    out = {"lambdas": list(lambdas), "n_runs": n_runs, "n_mcs": n_mcs, "interval": interval, "modes": []}
    for mi, (mode, s, k) in enumerate(modes):
        curves, speed, ms = autocorrelation_curves(lambdas, n_runs, n_mcs, interval, mode, s or 2, k or 1,
                                                   id0=mi * 100000, device=device)
        name = "serial" if mode == "serial" else f"parallel s={s} k={k}"
        say(f"{name}: A(1) per lambda {np.round(curves[:, 1], 3).tolist()}, {ms / 1e3:.1f} s")
        out["modes"].append({"mode": name, "A": curves.tolist(), "mean_speed": speed.tolist(), "ms": ms})
    return out
