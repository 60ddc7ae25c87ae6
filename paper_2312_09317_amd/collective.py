"""Polar order of a persistent 3D cell collective against cell density
(Results, motility models; Fig. 5C; 3D model settings table).

Cells of V_target 150 are packed at a given density into a periodic L^3
lattice (inputs.collective_3d) and advanced with the persistence term
(eq. 5, direction update eq. 6) for n_mcs MCS.  The order index is the
length of the mean of the cells' unit persistence directions: near 0 when
cells move independently, near 1 when the collective moves as one.  The
paper reports a sharp rise of the order index around density 0.5 when the
scheme preserves the serial CPM's update statistics, and its loss when a
thread runs all of its area's attempts back to back (k = s^d).
"""
import numpy as np

from . import cpm, inputs


def order_index(sim) -> float:
    """|mean unit direction| over the cells whose direction is set."""
    P = sim.persistence().cpu().numpy()[1:].astype(np.float64)
    norm = np.linalg.norm(P, axis=1)
    alive = norm > 0
    if not alive.any():
        return 0.0
    u = P[alive] / norm[alive, None]
    return float(np.linalg.norm(u.mean(axis=0)))


def order_vs_density(densities, L=128, n_mcs=2000, runs=3, s=2, k=1, seed0=1, device="cuda", log=None):
    """Order index after n_mcs MCS per density (mean and standard deviation
    over `runs` runs with different seeds), cells per run, and the GPU
    milliseconds of the sweeps."""
    import torch
    say = log or (lambda m: None)
    rows = []
    total_ms, total_sites = 0.0, 0
    for d in densities:
        vals, cells = [], 0
        for r in range(runs):
            w = inputs.collective_3d(L=L, density=d, seed=seed0 + r, n_mcs=n_mcs)
            p = cpm.Params.from_workload(w, sub=s, attempts=k, lattice_id=r)
            sim = cpm.Simulation(p, w.lattice, w.cell_type, device=device)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sim.sweep(n_mcs)
            e1.record()
            torch.cuda.synchronize()
            total_ms += e0.elapsed_time(e1)
            total_sites += w.n_sites * n_mcs
            vals.append(order_index(sim))
            cells = w.n_cells
            sim.close()
        rows.append({"density": float(w.extra["density"]), "requested": float(d), "cells": int(cells),
                     "order_mean": float(np.mean(vals)), "order_sd": float(np.std(vals)), "runs": vals})
        say(f"s={s} k={k} density {w.extra['density']:.3f} ({cells} cells): order {np.mean(vals):.3f} "
            f"+- {np.std(vals):.3f}")
    return {"L": L, "n_mcs": n_mcs, "runs": runs, "s": s, "k": k, "rows": rows, "ms": total_ms,
            "attempts": total_sites}
