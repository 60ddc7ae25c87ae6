"""Speed against accuracy of the parallel scheme (Results, motility models;
Fig. 5A, Fig. 6E).

An ensemble is n_runs copies of one workload that differ only in their
lattice id (so in their random numbers), advanced together as one batch.
The reference ensemble runs the serial CPM (cpm_batch_sweep_serial), the
others the parallel scheme at a given sub-area edge s and attempts per
activation k.  After n_mcs MCS the library counts, per pixel, the runs whose
lattice holds a cell there (cpm_batch_occupancy).  Agreement is measured as
in the paper: per-pixel binary cross-entropy, in bits, of the serial
occupancy p against the parallel occupancy q (clipped to [1/(2n), 1 -
1/(2n)] for n parallel runs), averaged over pixels; accuracy = 1 - that
mean.  A second serial ensemble scored the same way gives the accuracy that
ensembles of this size reach when the scheme is exact (the noise floor).
"""
import numpy as np

from . import cpm


def run_ensemble(w, n_runs, n_mcs, mode="parallel", s=None, k=None, id0=0, device="cuda"):
    """Occupancy counts (int64 numpy, one per pixel) of an ensemble after
    n_mcs MCS, the GPU milliseconds the sweeps took, and the attempt
    statistics summed over runs.  mode: "parallel" (at s, k; the workload's
    own when None) or "serial"."""
    import torch
    over = {}
    if s is not None:
        over["sub"] = int(s)
    if k is not None:
        over["attempts"] = int(k)
    params = [cpm.Params.from_workload(w, lattice_id=id0 + r, **over) for r in range(n_runs)]
    b = cpm.Batch(params, [w.lattice] * n_runs, [w.cell_type] * n_runs,
                  [w.act] * n_runs if w.lambda_act is not None else None, device=device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if mode == "parallel":
        b.sweep(1)  # the first call captures the MCS graph: keep it out of the timing
        n_run = n_mcs - 1
    else:
        n_run = n_mcs
    e0.record()
    if mode == "parallel":
        b.sweep(n_run)
    else:
        b.sweep_serial(n_run)
    e1.record()
    occ = b.occupancy()
    torch.cuda.synchronize()
    stats = np.asarray(b.attempt_stats(), dtype=np.int64).sum(axis=0)
    counts = occ.cpu().numpy().astype(np.int64)
    ms = e0.elapsed_time(e1)
    b.close()
    return counts, ms, stats, n_run


def cross_entropy_bits(counts_ref, n_ref, counts_par, n_par):
    """Mean per-pixel cross-entropy (bits) of the reference occupancy against
    the parallel one, the latter clipped to [1/(2 n_par), 1 - 1/(2 n_par)]."""
    p = np.asarray(counts_ref, dtype=np.float64) / n_ref
    eps = 1.0 / (2.0 * n_par)
    q = np.clip(np.asarray(counts_par, dtype=np.float64) / n_par, eps, 1.0 - eps)
    return float(np.mean(-(p * np.log2(q) + (1.0 - p) * np.log2(1.0 - q))))


def study(w, configs, n_runs=250, n_mcs=200, device="cuda", log=None):
    """Accuracy and speed of the parallel scheme at each (s, k) in configs
    against a serial reference ensemble of the workload w."""
    say = log or (lambda m: None)
    ref, ref_ms, ref_stats, ref_mcs = run_ensemble(w, n_runs, n_mcs, "serial", id0=0, device=device)
    say(f"serial reference: {n_runs} runs x {n_mcs} MCS in {ref_ms / 1e3:.1f} s")
    floor, _, _, _ = run_ensemble(w, n_runs, n_mcs, "serial", id0=n_runs, device=device)
    out = {"n_runs": n_runs, "n_mcs": n_mcs,
           "serial": {"ms_per_mcs": ref_ms / ref_mcs,
                      "attempts_per_s": n_runs * w.n_sites * ref_mcs / (ref_ms / 1e3)},
           "noise_floor_accuracy": 1.0 - cross_entropy_bits(ref, n_runs, floor, n_runs),
           "reference_entropy_bits": float(np.mean(_entropy(ref / n_runs))),
           "parallel": []}
    for c, (s, k) in enumerate(configs):
        par, ms, stats, n_run = run_ensemble(w, n_runs, n_mcs, "parallel", s=s, k=k,
                                             id0=(c + 2) * n_runs, device=device)
        acc = 1.0 - cross_entropy_bits(ref, n_runs, par, n_runs)
        rate = n_runs * w.n_sites * n_run / (ms / 1e3)
        say(f"s={s} k={k}: accuracy {acc:.4f}, {rate:.3e} attempts/s")
        out["parallel"].append({"s": s, "k": k, "accuracy": acc, "attempts_per_s": rate,
                                "ms_per_mcs": ms / n_run,
                                "accepted_per_attempt": float(stats[2]) / max(1, int(stats[0]))})
    return out


def _entropy(p):
    p = np.asarray(p, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        h = -(p * np.log2(p) + (1 - p) * np.log2(1 - p))
    return np.nan_to_num(h)
