"""Benchmark: site copy-attempts per second of the CPM sweep on one MI355X.

Workload: 3D 256^3 periodic lattice, 19,683 cells seeded as 8^3 cubes on a
jittered 27^3 grid, Moore-26 neighbourhood, J(cell,cell)=40, J(cell,medium)=20,
lambda_V=25, V_target=500, lambda_S=0.5, S_target=2690, T=20, checkerboard
scheme with s=2 (4^3 thread areas, 2x2x2 colours), k=1, Philox seed 1.

One step = one Monte Carlo step (MCS) = 256^3 copy attempts = 64
activations.  W warm-up steps, then K timed steps (default K=1000, the full
1000-MCS run), bracketed by device synchronisation; the tracked cell
volumes / surfaces are recounted from the lattice once at the end of the
timed region.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  Also reports the roofline position of the dominant
kernel (the activation kernel) and the CPU oracle's throughput on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "site copy-attempts/s on 3D 256³ (HBM % peak); emulator vs CPM cost per point"
HBM_PEAK_GBS = 8000.0

# HBM-side bytes per activation launch of each workload's activation kernel,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch) scaled by
# what the same counters read for a plain 256 MiB copy (FETCH x 2.0, WRITE x
# 1.0), for the kernel sources whose sha256 prefix is given and the tiling
# the counters were taken with; reported only while both are unchanged.
KERNEL_SOURCES = ("cpm_sweep_kernels.hpp", "cpm_sweep_inst.hip", "cpm_sweep.hip", "cpm_device.hpp", "cpm_internal.hpp")
_SHA = "0d1c5c1761aed574"
# 3D 256^3 (16-bit labels, in place)
MEASURED_TRAFFIC = {"sources_sha256": _SHA, "layout": "in_place", "tile": [64, 2, 2], "order": "linear",
                    "fetch_kib": 15132.7, "write_kib": 384.6, "fetch_scale": 2.0, "write_scale": 1.0}
# 1024^3 tissue (label-type-activity words)
MEASURED_TRAFFIC_TISSUE = {"sources_sha256": _SHA, "layout": "in_place", "tile": [256, 1, 1], "order": "linear",
                           "fetch_kib": 1807049.8, "write_kib": 255437.1, "fetch_scale": 2.0, "write_scale": 1.0}
# 2048^2 sorting (16-bit labels)
MEASURED_TRAFFIC_SORTING = {"sources_sha256": _SHA, "layout": "in_place", "tile": [256, 1, 1], "order": "linear",
                            "fetch_kib": 4258.5, "write_kib": 244.8, "fetch_scale": 2.0, "write_scale": 1.0}
# 256^3 collective (16-bit labels, persistence term)
MEASURED_TRAFFIC_COLLECTIVE = {"sources_sha256": _SHA, "layout": "in_place", "tile": [64, 2, 2], "order": "linear",
                               "fetch_kib": 16776.5, "write_kib": 3848.2, "fetch_scale": 2.0, "write_scale": 1.0}
# 512 uneven 2D lattices (16-bit label-activity words; in place, the
# library's tiles, graph replay)
MEASURED_TRAFFIC_BATCH = {"sources_sha256": _SHA, "layout": "in_place", "tile": None, "order": "linear",
                          "fetch_kib": 56122.4, "write_kib": 10233.0, "fetch_scale": 2.0, "write_scale": 1.0}


def kernel_sources_sha():
    """sha256 prefix of the activation kernels' sources, as the traffic tables record it."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_09317_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic_bytes(layout=None, table=None, tile=None, order=None):
    """HBM bytes per launch of a traffic table, or None when the kernel
    sources, the layout, the tile shape or the tile order differ from those
    the counters were taken on."""
    t = MEASURED_TRAFFIC if table is None else table
    if kernel_sources_sha() != t["sources_sha256"] or (layout is not None and layout != t["layout"]):
        return None
    if tile is not None and t.get("tile") is not None and list(tile) != list(t["tile"]):
        return None
    if order is not None and order != t.get("order", "linear"):
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def bytes_per_attempt(ndim, s, k, p_acc, act=False):
    # per activation each thread area stages the halo box of its active
    # sub-area, (s+2)^d int32 sites, which at s = 2 is the whole (2s)^d area,
    # and writes back its accepted copy; with the Act term the uint8 activity
    # of the same sites as well
    f = min(1.0, (s + 2.0) / (2.0 * s)) ** ndim
    b = 4.0 * f * (2 * s) ** ndim / k + 4.0 * p_acc
    if act:
        b += 1.0 * f * (2 * s) ** ndim / k + 1.0 * p_acc
    return b


def host_cpus():
    """CPUs of the host (nproc) and those this process may run on."""
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count()
    return {"nproc": os.cpu_count(), "allowed": allowed}


def pinned(fn):
    """fn() with the process pinned to one CPU, as taskset -c would pin it;
    returns (fn's result, the CPU)."""
    try:
        old = os.sched_getaffinity(0)
        cpu = max(old)
        os.sched_setaffinity(0, {cpu})
    except (AttributeError, OSError):
        return fn(), None
    try:
        return fn(), cpu
    finally:
        os.sched_setaffinity(0, old)


def oracle_model(w):
    import oracle
    return oracle.Model(w.ndim, w.dims[:w.ndim], w.J, w.lambda_V, w.V_target, w.lambda_S, w.S_target,
                        lambda_act=w.lambda_act, max_act=w.max_act, T=w.T, seed=w.seed, lattice_id=w.lattice_id,
                        s=w.s, k=w.k, obstacle_type=w.obstacle_type, lambda_P=w.lambda_P, mu_P=w.mu_P,
                        dt_P=w.dt_P, lambda_C=w.lambda_C, C_field=w.C_field)


def cpu_baseline(w, n_mcs):
    """The oracle, pinned to one CPU, on the first n_mcs MCS of workload w."""
    import oracle
    st = oracle.State(oracle_model(w), w.lattice, w.cell_type, w.act)

    def run():
        t0 = time.perf_counter()
        st.sweep(n_mcs)
        return time.perf_counter() - t0
    dt, cpu = pinned(run)
    attempts = int(st.stats[0])
    return {"value": attempts / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_mcs} MCS of the same {w.name} workload ({attempts} attempts, "
                      f"{dt:.1f} s, one thread pinned to CPU {cpu}, initial recount excluded)",
            "host_cpus": host_cpus(), "pinned_cpu": cpu, "p_acc": float(st.stats[2]) / max(1, attempts)}


def cpu_fields(cpu):
    """The cpu_baseline object of a bench line."""
    if not cpu:
        return None
    return {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample", "host_cpus", "pinned_cpu") if k in cpu}


def cpu_baseline_pool(ws, n_mcs, threads):
    """The oracle on lattices ws (n_mcs MCS each), on one thread and then on
    `threads` threads (the oracle's C calls release the GIL, so each thread
    runs its own lattices on its own core)."""
    import concurrent.futures
    import oracle

    def run(group):
        n = 0
        for w in group:
            st = oracle.State(oracle_model(w), w.lattice, w.cell_type, w.act)
            st.sweep(n_mcs)
            n += int(st.stats[0])
        return n

    def timed(fn):
        t0 = time.perf_counter()
        n = fn()
        return n, time.perf_counter() - t0
    (n1, dt1), cpu = pinned(lambda: timed(lambda: run(ws)))
    groups = [ws[i::threads] for i in range(threads)]
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as pool:
        nn, dtn = timed(lambda: sum(pool.map(run, groups)))
    return ({"value": n1 / dt1, "unit": "attempts/s", "cores": 1, "kind": "oracle",
             "sample": f"{len(ws)} lattices x {n_mcs} MCS of the same workload ({n1} attempts, {dt1:.1f} s, one "
                       f"thread pinned to CPU {cpu})", "host_cpus": host_cpus(), "pinned_cpu": cpu},
            {"value": nn / dtn, "unit": "attempts/s", "cores": threads, "kind": "oracle",
             "sample": f"the same {len(ws)} lattices x {n_mcs} MCS on {threads} threads ({dtn:.1f} s)"})


def sample_mcs(args, default):
    """MCS of the oracle sample: --cpu-mcs, else the workload's default."""
    return default if args.cpu_mcs is None else args.cpu_mcs


def copy_calibration(nbytes):
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reads_per_copy": nbytes, "writes_per_copy": nbytes, "copies": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-mcs", type=int, default=None,
                    help="MCS of the oracle sample (0 to skip; default: about 10-15 s of oracle work per "
                         "workload: 6 for the 256^3 sweep, 120 for sorting, 2 for the collective)")
    ap.add_argument("--workload", choices=("sweep", "tissue", "sorting", "collective", "collective-order", "accuracy",
                                           "polarisation", "batch", "emulator"),
                    default="sweep",
                    help="sweep: the 3D 256^3 benchmark (default); tissue: 3D 1024^3 with obstacles and the "
                         "Act term; sorting: 2D 2048^2 two-type cell sorting; collective: 3D 256^3 packed "
                         "collective with the persistence term; collective-order: polar order of the 3D "
                         "collective after --order-mcs MCS against cell density, k = 1 and k = s^d; "
                         "accuracy: speed and accuracy of the parallel "
                         "scheme against the serial CPM (2D circular chemotaxis ensembles); polarisation: "
                         "directional autocorrelation of Act cells, serial CPM vs parallel scheme; batch: 512 uneven "
                         "2D lattices; emulator: "
                         "train the emulator on batched runs and score it against fresh ones")
    ap.add_argument("--layout", default="tune", choices=("tune", "auto", "box", "full_rows", "in_place"),
                    help="sweep layout: tune = time the candidates first and take the fastest (default)")
    ap.add_argument("--tile", default=None,
                    help="thread areas per workgroup tile as X,Y,Z (with a named --layout; default: the "
                         "library's choice)")
    ap.add_argument("--tile-order", default="auto", choices=("auto", "linear", "bricks"),
                    help="with a named --layout: the order in which each XCD takes its tiles")
    ap.add_argument("--tune-mcs", type=int, default=6, help="MCS timed per candidate layout when tuning")
    ap.add_argument("--batch-n", type=int, default=512, help="batch workload: lattices (512 in the benchmark)")
    ap.add_argument("--batch-max-side", type=int, default=512,
                    help="batch workload: largest side (512 in the benchmark; 64 gives a batch of 64^2 lattices "
                         "whose MCS time is mostly launch or barrier overhead)")
    ap.add_argument("--batch-mode", default=None, choices=("graph", "eager", "persistent"),
                    help="batch workload: how each sweep is launched (default: the tuner's choice, else graph)")
    ap.add_argument("--order-densities", default="0.1,0.2,0.3,0.4,0.5,0.6,0.7,0.8,0.9",
                    help="collective-order workload: cell densities")
    ap.add_argument("--order-side", type=int, default=128, help="collective-order workload: lattice side")
    ap.add_argument("--order-mcs", type=int, default=2000, help="collective-order workload: MCS per run")
    ap.add_argument("--order-runs", type=int, default=3, help="collective-order workload: runs per density")
    ap.add_argument("--acc-runs", type=int, default=250, help="accuracy workload: runs per ensemble")
    ap.add_argument("--acc-mcs", type=int, default=200, help="accuracy workload: MCS per run")
    ap.add_argument("--emu-train", type=int, default=8192, help="emulator workload: training runs")
    ap.add_argument("--emu-train-reps", type=int, default=1,
                    help="emulator workload: runs per training point (the emulator learns their mean)")
    ap.add_argument("--emu-test", type=int, default=256, help="emulator workload: held-out points")
    ap.add_argument("--emu-reps", type=int, default=8, help="emulator workload: replicates per held-out point")
    ap.add_argument("--emu-epochs", type=int, default=2000)
    ap.add_argument("--emu-data", default=None, help="emulator workload: .npz of the study's CPM runs "
                    "(written if missing, reused if present)")
    ap.add_argument("--emu-lr", type=float, default=1e-3)
    ap.add_argument("--emu-batch", type=int, default=256)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes, 5 times (calibrates "
                         "the HBM byte counters of a profiler against a known traffic)")
    args = ap.parse_args()
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1"}))
        log("bench.py runs on one GPU only: the sweep is not sharded across GPUs")
        sys.exit(2)

    import torch
    from paper_2312_09317_amd import cpm, inputs

    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "tissue":
        return bench_tissue(args)
    if args.workload == "sorting":
        return bench_sorting(args)
    if args.workload == "collective":
        return bench_collective(args)
    if args.workload == "collective-order":
        return bench_collective_order(args)
    if args.workload == "accuracy":
        return bench_accuracy(args)
    if args.workload == "polarisation":
        return bench_polarisation(args)
    if args.workload == "emulator":
        return bench_emulator(args)
    w = inputs.config1(n_mcs=args.steps)
    log(f"workload {w.name}: {w.n_sites} sites, {w.n_cells} cells")
    params, tuning = choose_layout(args, cpm, cpm.Params.from_workload(w), w)
    sim = cpm.Simulation(params, w.lattice, w.cell_type, device="cuda:0")
    torch.cuda.synchronize()
    sim.sweep(args.warmup)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} MCS)")
    att0 = sim.attempt_stats()

    n_act = (2 * w.s) ** w.ndim // w.k
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev2 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    sim.sweep(args.steps)
    ev1.record()
    v, s, c = sim.cell_stats(centroids=True)
    ev2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep_ms = ev0.elapsed_time(ev1)
    total_ms = ev0.elapsed_time(ev2)
    log(f"timed {args.steps} MCS: {total_ms:.1f} ms (sweep {sweep_ms:.1f} ms, wall {wall * 1e3:.1f} ms)")

    # sanity: tracked counters equal the recount
    tv, ts = sim.counters()
    torch.cuda.synchronize()
    if not (torch.equal(tv[1:], v[1:]) and torch.equal(ts[1:], s[1:])):
        log("ERROR: tracked counters differ from the lattice recount")
        sys.exit(3)

    attempts = args.steps * w.n_sites
    value = attempts / (total_ms / 1e3)
    # accepted copies per attempt of the timed region, from the kernels' own counts
    att1 = sim.attempt_stats()
    p_acc = (att1[2] - att0[2]) / max(1, att1[0] - att0[0])
    n_cpu = sample_mcs(args, 6)
    cpu = cpu_baseline(w, n_cpu) if n_cpu > 0 else None
    launches = args.steps * n_act
    # the activation kernels run back to back on one stream: the timed
    # region's time per launch is their average duration (the MCS loop
    # launches nothing else in this workload, and the two 16-bit copy passes
    # per call are under 0.05% of the region at 1000 MCS)
    avg_launch_s = (sweep_ms / 1e3) / launches
    per_launch_bytes = bytes_per_attempt(w.ndim, w.s, w.k, p_acc) * (w.n_sites // n_act)
    achieved = per_launch_bytes / avg_launch_s / 1e9
    tiling = cpm.cpm_tile_shape(params, w.n_cells)
    traffic = measured_traffic_bytes(tiling["layout"], tile=tiling["areas"], order=tiling["order"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.dims), "n_cells": w.n_cells, "sub": w.s,
                   "attempts_per_activation": w.k, "mcs_per_step": 1, "activations_per_mcs": n_act,
                   "temperature": w.T, "seed": w.seed, "tiling": tiling,
                   "label_storage": label_storage(tiling), "energy_arithmetic": "int64, 2^-16 fixed point",
                   "tuning_ms_per_mcs": tuning},
        "roofline": roofline_fields(achieved, traffic, avg_launch_s, "tile_sweep_kernel",
                                    bytes_per_attempt(w.ndim, w.s, w.k, p_acc)),
        "cpu_baseline": cpu_fields(cpu),
    }
    print(json.dumps(out), flush=True)
    sim.close()


def traffic_of(cpm, params, w, table):
    """A traffic table's bytes per launch when the model's tiling is the one
    the counters were taken with."""
    t = cpm.cpm_tile_shape(params, w.n_cells)
    return measured_traffic_bytes(t["layout"], table, tile=t["areas"], order=t["order"])


def label_storage(tiling, act_words=False):
    """What the activation kernel reads per site, for the report."""
    if act_words:
        return "uint32 words: label + 1, type and activity, written over the int32 lattice during a sweep"
    if tiling.get("labels16"):
        return "uint16 mirror (label + 1) of the int32 lattice"
    return "int32 labels"


def roofline_fields(achieved_gbs, traffic, avg_launch_s, kernel, bpa):
    """The roofline object: `frac` from the algorithmic bytes (the staged
    scheme's int32 sites per attempt) and, beside it, the fraction the
    measured HBM-side bytes per launch give at the same launch time."""
    real = traffic / avg_launch_s / 1e9 if traffic else None
    return {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": traffic,
            "achieved_measured_bytes": real, "frac_measured_bytes": real / HBM_PEAK_GBS if real else None,
            "kernel": kernel, "avg_launch_us": avg_launch_s * 1e6, "bytes_per_attempt": bpa,
            "byte_model": "algorithmic: the staged scheme's int32 halo sites (+ uint8 activity) per attempt; "
                          "the in-place kernels read the stored words where they lie, so frac can pass 1 while "
                          "frac_measured_bytes (HBM-side bytes from the profiler's counters) stays below it"}


def choose_layout(args, cpm, params, w):
    """The sweep layout: timed candidates (--layout tune) or the one named."""
    if args.layout != "tune":
        tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else (0, 0, 0)
        return params.replace(layout=args.layout, tile=tile, tile_order=args.tile_order), None
    r = cpm.autotune(params, w.lattice, w.cell_type, w.act, trial_mcs=args.tune_mcs)
    name = lambda k: f"{k[0]}{list(k[1])}" + ("/bricks" if k[2] == "bricks" else "")
    log("autotune (ms per MCS): " + ", ".join(f"{name(k)}: {v:.3f}" for k, v in sorted(r["times"].items(), key=lambda kv: kv[1])))
    lay, tile, order = r["best"]
    return (params.replace(layout=lay, tile=tile, tile_order=order),
            {name(k): round(v, 4) for k, v in r["times"].items()})


def bench_tissue(args):
    """1024^3 lattice (4 GiB of int32 labels, too many cells for the 16-bit
    copy) with Gaussian-random-field obstacles, ~820k cells of V_target
    1000, half of them motile with the Act term.  Step = 1 MCS = 64
    activations; nothing of it fits in the caches."""
    import torch
    from paper_2312_09317_amd import cpm, inputs
    t0 = time.perf_counter()
    w = inputs.config2(n_mcs=args.steps)
    log(f"workload {w.name}: {w.n_sites} sites, {w.n_cells} cells, built in {time.perf_counter() - t0:.1f} s")
    params, tuning = choose_layout(args, cpm, cpm.Params.from_workload(w), w)
    sim = cpm.Simulation(params, w.lattice, w.cell_type, w.act, device="cuda:0")
    del w.lattice, w.act
    sim.sweep(args.warmup)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    sim.sweep(args.steps)
    e1.record()
    v, s, _ = sim.cell_stats(centroids=False)
    e2.record()
    torch.cuda.synchronize()
    sweep_ms, total_ms = e0.elapsed_time(e1), e0.elapsed_time(e2)
    tv, ts = sim.counters()
    torch.cuda.synchronize()
    if not (torch.equal(tv[1:], v[1:]) and torch.equal(ts[1:], s[1:])):
        log("ERROR: tracked counters differ from the lattice recount")
        sys.exit(3)
    n_act = (2 * w.s) ** w.ndim // w.k
    att = sim.attempt_stats()
    p_acc = att[2] / max(1, att[0])
    avg_launch_s = sweep_ms / 1e3 / (args.steps * n_act)
    per_launch_bytes = bytes_per_attempt(3, w.s, w.k, p_acc, act=True) * (w.n_sites // n_act)
    achieved = per_launch_bytes / avg_launch_s / 1e9
    cpu = None
    n_cpu = sample_mcs(args, 72)
    if n_cpu > 0:
        # the oracle on a 128^3 crop of the same recipe (obstacle field, cells
        # of V_target 1000 at the same density, half of them motile)
        crop = inputs.config2(L=128, grid=12, n_mcs=n_cpu)
        cpu = cpu_baseline(crop, n_cpu)
        cpu["sample"] = f"128^3 crop of the recipe ({crop.n_cells} cells): " + cpu["sample"]
    print(json.dumps({
        "metric": "site copy-attempts/s on 3D 1024³ tissue (HBM % peak)",
        "value": w.n_sites * args.steps / (total_ms / 1e3), "unit": "attempts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.dims), "n_cells": w.n_cells,
                   "obstacle_voxels": w.extra["obstacle_voxels"], "sub": w.s, "attempts_per_activation": w.k,
                   "act": True, "tiling": cpm.cpm_tile_shape(params, w.n_cells), "tuning_ms_per_mcs": tuning,
                   "label_storage": label_storage(None, act_words=True)},
        "roofline": roofline_fields(achieved, traffic_of(cpm, params, w, MEASURED_TRAFFIC_TISSUE), avg_launch_s,
                                    "tile_sweep_kernel_packed", bytes_per_attempt(3, w.s, w.k, p_acc, act=True)),
        "cpu_baseline": cpu_fields(cpu)}), flush=True)
    sim.close()


def bench_sorting(args):
    """Two-type cell sorting on a 2048^2 lattice (1,600 cells of 50 x 50,
    differential adhesion), the paper's 2D benchmark workload.  Step = 1 MCS
    = 16 activations.  Also reports the homotypic share of cell-cell contacts
    before and after the timed MCS (it grows as the populations sort)."""
    import numpy as np
    import torch
    from paper_2312_09317_amd import cpm, inputs
    w = inputs.sorting_2d(n_mcs=args.steps)
    log(f"workload {w.name}: {w.n_sites} sites, {w.n_cells} cells")
    params, tuning = choose_layout(args, cpm, cpm.Params.from_workload(w), w)
    sim = cpm.Simulation(params, w.lattice, w.cell_type, device="cuda:0")
    def homotypic():
        m = sim.contacts().cpu().numpy()
        return float(np.trace(m[1:, 1:]) / max(1, m[1:, 1:].sum()))
    h0 = homotypic()
    sim.sweep(args.warmup)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    sim.sweep(args.steps)
    e1.record()
    v, s, _ = sim.cell_stats(centroids=False)
    e2.record()
    torch.cuda.synchronize()
    sweep_ms, total_ms = e0.elapsed_time(e1), e0.elapsed_time(e2)
    h1 = homotypic()
    n_act = (2 * w.s) ** w.ndim // w.k
    att = sim.attempt_stats()
    p_acc = att[2] / max(1, att[0])
    avg_launch_s = sweep_ms / 1e3 / (args.steps * n_act)
    per_launch_bytes = bytes_per_attempt(2, w.s, w.k, p_acc) * (w.n_sites // n_act)
    achieved = per_launch_bytes / avg_launch_s / 1e9
    n_cpu = sample_mcs(args, 120)
    cpu = cpu_baseline(w, n_cpu) if n_cpu > 0 else None
    print(json.dumps({
        "metric": "site copy-attempts/s on 2D 2048² cell sorting", "value": w.n_sites * args.steps / (total_ms / 1e3),
        "unit": "attempts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.dims), "n_cells": w.n_cells, "sub": w.s,
                   "attempts_per_activation": w.k, "tiling": cpm.cpm_tile_shape(params, w.n_cells),
                   "tuning_ms_per_mcs": tuning, "homotypic_contacts_before": h0,
                   "homotypic_contacts_after": h1, "mcs_run": args.warmup + args.steps},
        "roofline": roofline_fields(achieved, traffic_of(cpm, params, w, MEASURED_TRAFFIC_SORTING), avg_launch_s,
                                    "tile_sweep_kernel", bytes_per_attempt(2, w.s, w.k, p_acc)),
        "cpu_baseline": cpu_fields(cpu)}),
        flush=True)
    sim.close()


def bench_collective(args):
    """A packed 3D collective of persistently moving cells on a 256^3
    lattice (54,872 cells of V_target 150 at density 0.49; 16-bit labels),
    the paper's 3D collective settings (mu 0.95, dt 15, lambda_persistence
    40).  Step = 1 MCS = 64 activations plus the direction update (centroid
    sums of every cell, then one thread per cell).  Also reports the polar
    order of the cells' directions, |sum of unit directions| / cells."""
    import numpy as np
    import torch
    from paper_2312_09317_amd import cpm, inputs
    w = inputs.collective_3d(n_mcs=args.steps)
    log(f"workload {w.name}: {w.n_sites} sites, {w.n_cells} cells, density {w.extra['density']:.3f}")
    # centroids recounted at each direction update (the library's default;
    # keeping them in the sweeps instead measured slower here: 0.965 against
    # 0.870 ms per MCS, six 64-bit atomics per accepted copy at 8.4% acceptance)
    params, tuning = choose_layout(args, cpm, cpm.Params.from_workload(w), w)
    sim = cpm.Simulation(params, w.lattice, w.cell_type, device="cuda:0")

    def order():
        P = sim.persistence().cpu().numpy()[1:].astype(np.float64)
        alive = np.any(P != 0, axis=1)
        return float(np.linalg.norm(P[alive].sum(axis=0)) / (16384.0 * max(1, alive.sum())))
    sim.sweep(args.warmup)
    torch.cuda.synchronize()
    o0 = order()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    sim.sweep(args.steps)
    e1.record()
    v, s, _ = sim.cell_stats(centroids=False)
    e2.record()
    torch.cuda.synchronize()
    sweep_ms, total_ms = e0.elapsed_time(e1), e0.elapsed_time(e2)
    o1 = order()
    tv, ts = sim.counters()
    torch.cuda.synchronize()
    if not (torch.equal(tv[1:], v[1:]) and torch.equal(ts[1:], s[1:])):
        log("ERROR: tracked counters differ from the lattice recount")
        sys.exit(3)
    n_act = (2 * w.s) ** w.ndim // w.k
    att = sim.attempt_stats()
    p_acc = att[2] / max(1, att[0])
    # the timed region also holds one direction update per MCS, so this
    # average is an upper bound on the activation kernel's duration
    avg_launch_s = sweep_ms / 1e3 / (args.steps * n_act)
    per_launch_bytes = bytes_per_attempt(3, w.s, w.k, p_acc) * (w.n_sites // n_act)
    achieved = per_launch_bytes / avg_launch_s / 1e9
    n_cpu = sample_mcs(args, 2)
    cpu = cpu_baseline(w, n_cpu) if n_cpu > 0 else None
    print(json.dumps({
        "metric": "site copy-attempts/s on a 3D 256³ persistent cell collective",
        "value": w.n_sites * args.steps / (total_ms / 1e3), "unit": "attempts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.dims), "n_cells": w.n_cells,
                   "density": w.extra["density"], "sub": w.s, "attempts_per_activation": w.k,
                   "persistence": {"lambda": float(w.lambda_P[1]), "mu": float(w.mu_P[1]), "dt": w.dt_P,
                                   "centroids": "recount"},
                   "tiling": cpm.cpm_tile_shape(params, w.n_cells), "tuning_ms_per_mcs": tuning,
                   "order_before": o0, "order_after": o1, "mcs_run": args.warmup + args.steps},
        "roofline": roofline_fields(achieved, traffic_of(cpm, params, w, MEASURED_TRAFFIC_COLLECTIVE), avg_launch_s,
                                    "tile_sweep_kernel", bytes_per_attempt(3, w.s, w.k, p_acc)),
        "cpu_baseline": cpu_fields(cpu)}),
        flush=True)
    sim.close()


def bench_accuracy(args):
    """Speed against accuracy (Fig. 6E): ensembles of the 2D circular
    chemotaxis workload (256^2, 8 cells of 50^2, lambda_chemotaxis 10), one
    serial reference ensemble and one parallel ensemble per (s, k), each of
    --acc-runs runs of --acc-mcs MCS advanced as one batch; accuracy = 1 -
    mean pixel cross-entropy of the serial occupancy against the parallel
    one.  value: attempts/s of the parallel ensemble at the default s = 2,
    k = 1."""
    from paper_2312_09317_amd import accuracy, inputs
    w = inputs.chemotaxis_2d(n_mcs=args.acc_mcs)
    configs = [(1, 1), (2, 1), (2, 4), (4, 1), (4, 8), (8, 1), (8, 8)]
    log(f"workload {w.name}: {args.acc_runs} runs per ensemble, {args.acc_mcs} MCS, (s, k) in {configs}")
    out = accuracy.study(w, configs, n_runs=args.acc_runs, n_mcs=args.acc_mcs, log=log)
    main_row = next(r for r in out["parallel"] if (r["s"], r["k"]) == (2, 1))
    cpu = None
    if sample_mcs(args, 1) > 0:
        # the oracle runs an ensemble sample of the same shape: 32 runs of
        # the parallel scheme at s = 2, k = 1 over --acc-mcs MCS
        import oracle
        m = oracle.Model(w.ndim, w.dims[:w.ndim], w.J, w.lambda_V, w.V_target, w.lambda_S, w.S_target,
                         T=w.T, seed=w.seed, s=w.s, k=w.k, lambda_C=w.lambda_C, C_field=w.C_field)
        t0 = time.perf_counter()
        oracle.replicates(m, w.lattice, w.cell_type, args.acc_mcs, 32, mode="dcs")
        dt = time.perf_counter() - t0
        n_att = 32 * args.acc_mcs * w.n_sites
        cpu = {"value": n_att / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
               "sample": f"32 runs x {args.acc_mcs} MCS of the same workload at s = 2, k = 1 ({n_att} attempts, "
                         f"{dt:.1f} s, one thread)"}
    print(json.dumps({
        "metric": "site copy-attempts/s of a 2D chemotaxis ensemble, with its accuracy against the serial CPM",
        "value": main_row["attempts_per_s"], "unit": "attempts/s", "n_gpus": 1, "steps": args.acc_mcs,
        "warmup": 1, "ms_per_step": main_row["ms_per_mcs"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.dims), "n_cells": w.n_cells, "runs": args.acc_runs,
                   "study": out},
        "roofline": None,
        "cpu_baseline": cpu_fields(cpu)}),
        flush=True)


def bench_collective_order(args):
    """Order index of the persistent 3D collective after --order-mcs MCS
    against cell density (Fig. 5C): the parallel scheme at s = 2 with k = 1
    (update statistics kept) and with k = 8 = s^d (each thread's attempts
    back to back).  The line's value is the attempt rate over all runs."""
    from paper_2312_09317_amd import collective
    dens = [float(x) for x in args.order_densities.split(",")]
    modes = []
    for k in (1, 8):
        modes.append(collective.order_vs_density(dens, L=args.order_side, n_mcs=args.order_mcs,
                                                 runs=args.order_runs, s=2, k=k, log=log))
    ms = sum(m["ms"] for m in modes)
    att = sum(m["attempts"] for m in modes)
    print(json.dumps({
        "metric": "polar order index of a 3D persistent collective after N MCS, against cell density",
        "value": att / (ms / 1e3), "unit": "attempts/s", "n_gpus": 1, "steps": args.order_mcs, "warmup": 0,
        "ms_per_step": ms / (args.order_mcs * len(dens) * args.order_runs * len(modes)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"3d-{args.order_side}^3-collective-order", "mcs": args.order_mcs,
                   "runs": args.order_runs,
                   "modes": [{"s": m["s"], "k": m["k"],
                              "rows": [{kk: r[kk] for kk in ("density", "cells", "order_mean", "order_sd")}
                                       for r in m["rows"]]} for m in modes]},
        "roofline": None, "cpu_baseline": None}), flush=True)


def bench_polarisation(args):
    """Directional persistence of Act cells (Fig. 5B): single-cell 2D runs
    (200^2, one 50^2 cell, Max_act 50) at lambda_act 0..800, 50 runs each,
    750 MCS sampled every 50, under the serial CPM and the parallel scheme
    at (s, k) = (2, 1) and (2, 4); the directional autocorrelation A(lag) per
    lambda and mode.  value: attempts/s of the (2, 1) ensemble."""
    import numpy as np
    from paper_2312_09317_amd import polarisation
    lambdas = (0.0, 100.0, 200.0, 400.0, 800.0)
    out = polarisation.study(lambdas=lambdas, log=log)
    ser = np.asarray(out["modes"][0]["A"])
    rows = []
    for m in out["modes"]:
        A = np.asarray(m["A"])
        rows.append({"mode": m["mode"], "A_lag1": A[:, 1].round(4).tolist(), "A_lag3": A[:, 3].round(4).tolist(),
                     "max_abs_diff_vs_serial": float(np.abs(A - ser)[:, 1:].max()),
                     "mean_speed": np.round(m["mean_speed"], 4).tolist(), "gpu_s": m["ms"] / 1e3})
    n_att = len(lambdas) * out["n_runs"] * 200 * 200 * out["n_mcs"]
    main = out["modes"][1]
    cpu = None
    n_cpu = sample_mcs(args, 250)
    if n_cpu > 0:
        # the oracle on runs of the same ensemble: the parallel scheme at
        # s = 2, k = 1, lambda_act 400, ten lattice ids
        import oracle
        from paper_2312_09317_amd import inputs
        n1, dt, cpu_id = 0, 0.0, None
        for r in range(10):
            w = inputs.act_2d(lambda_act=400.0, n_mcs=n_cpu)
            w.lattice_id = r
            st = oracle.State(oracle_model(w), w.lattice, w.cell_type, w.act)

            def run():
                t0 = time.perf_counter()
                st.sweep(n_cpu)
                return time.perf_counter() - t0
            d, cpu_id = pinned(run)
            dt += d
            n1 += int(st.stats[0])
        cpu = {"value": n1 / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
               "sample": f"10 runs x {n_cpu} MCS of the same 200^2 Act cell at lambda_act 400, s = 2, k = 1 "
                         f"({n1} attempts, {dt:.1f} s, one thread pinned to CPU {cpu_id})",
               "host_cpus": host_cpus(), "pinned_cpu": cpu_id}
    print(json.dumps({
        "metric": "site copy-attempts/s of a 2D Act ensemble, with its directional autocorrelation against the serial CPM",
        "value": n_att / (main["ms"] / 1e3), "unit": "attempts/s", "n_gpus": 1, "steps": out["n_mcs"], "warmup": 0,
        "ms_per_step": main["ms"] / out["n_mcs"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "2d-200x200-act-single-cell", "lambdas": list(lambdas), "runs": out["n_runs"],
                   "interval": out["interval"], "modes": rows},
        "roofline": None, "cpu_baseline": cpu_fields(cpu)}), flush=True)


def bench_batch(args):
    """512 independent 2D lattices of uneven sizes (64..512, 30% cells, Act
    term, per-lattice parameters), advanced together: one launch per
    activation, each MCS one replay of a captured HIP graph.  Step = 1 MCS
    of every lattice."""
    import torch
    from paper_2312_09317_amd import cpm, inputs
    ws = inputs.config3(n_lattices=args.batch_n, seed=1, n_mcs=args.steps, L_max=args.batch_max_side)
    sites = sum(w.n_sites for w in ws)
    log(f"batch of {len(ws)} lattices, {sites} sites")
    params = [cpm.Params.from_workload(w) for w in ws]
    lattices, types = [w.lattice for w in ws], [w.cell_type for w in ws]
    cfg = {"layout": "in_place" if args.layout in ("tune", "auto") else args.layout, "tiles": ["auto"] * len(ws),
           "mode": args.batch_mode or "graph"}
    tuning = None
    if args.layout == "tune":
        r = cpm.autotune_batch(params, lattices, types, trial_mcs=args.tune_mcs, log=log)
        cfg = dict(r["best"], mode=args.batch_mode or r["best"]["mode"])
        tuning = {k: round(v, 4) for k, v in sorted(r["times"].items(), key=lambda kv: kv[1])}
    b = cpm.Batch(cpm.batch_params(params, cfg), lattices, types)
    b.launch_mode(cfg["mode"])
    classes = cpm.size_classes(params)
    tuned = {"layout": cfg["layout"], "mode": cfg["mode"],
             "tile_by_size_class": [{"sides": [min(ws[i].dims[0] for i in c), max(ws[i].dims[0] for i in c)],
                                     "lattices": len(c), "tile": cfg["tiles"][c[0]]} for c in classes]}
    log(f"batch configuration: {tuned}")
    b.sweep(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.sweep(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    n_act = (2 * ws[0].s) ** 2 // ws[0].k
    stats = b.attempt_stats()
    acc = float(sum(int(r[2]) for r in stats)) / max(1, sum(int(r[0]) for r in stats))
    avg_launch_s = ms / 1e3 / (args.steps * n_act)
    per_launch_bytes = bytes_per_attempt(2, ws[0].s, ws[0].k, acc, act=True) * (sites // n_act)
    achieved = per_launch_bytes / avg_launch_s / 1e9
    b.close()
    # measured traffic: taken in place with the library's tiles and graph replay
    default_cfg = cfg["layout"] == "in_place" and all(t == "auto" for t in cfg["tiles"]) and cfg["mode"] == "graph"
    batch_traffic = measured_traffic_bytes("in_place", MEASURED_TRAFFIC_BATCH) if default_cfg else None
    cpu = cpu_threads = None
    n_cpu = sample_mcs(args, 48)
    if n_cpu > 0:
        # the oracle on the first 64 lattices of the batch: one pinned
        # thread, then one thread per allowed CPU (at most 16)
        threads = max(1, min(16, host_cpus()["allowed"] or 1))
        cpu, cpu_threads = cpu_baseline_pool(ws[:64], n_cpu, threads)
    print(json.dumps({
        "metric": "site copy-attempts/s, 512 batched uneven 2D lattices", "value": sites * args.steps / (ms / 1e3),
        "unit": "attempts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"2d-batch-{len(ws)}-L64..{args.batch_max_side}", "n_lattices": len(ws), "sites": sites, "sub": ws[0].s,
                   "attempts_per_activation": ws[0].k, "act": True, "launch": tuned, "tuning_ms_per_mcs": tuning,
                   "label_storage": "uint16 words: label + 1 and activity (one cell type, at most 2,046 cells, "
                                    "Max_act <= 31), written from the int32 lattices and activities per sweep call"},
        "roofline": roofline_fields(achieved, batch_traffic, avg_launch_s, "batch_sweep_kernel",
                                    bytes_per_attempt(2, ws[0].s, ws[0].k, acc, act=True)),
        "cpu_baseline": cpu_fields(cpu), "cpu_baseline_threads": cpu_fields(cpu_threads)}), flush=True)


def bench_emulator(args):
    """The emulator study: batched CPM runs of the 512-lattice parameter
    space as training data, training on the GPU, and the held-out error
    against fresh CPM replicates, with the cost per parameter point of each."""
    from paper_2312_09317_amd import emulator
    r = emulator.study(n_train=args.emu_train, n_test=args.emu_test, reps=args.emu_reps, epochs=args.emu_epochs,
                       batch=args.emu_batch, lr=args.emu_lr, lr_final=args.emu_lr / 40, log=log,
                       data_path=args.emu_data, train_reps=args.emu_train_reps)
    cpu = emulator_cpu_baseline(args) if sample_mcs(args, 100) > 0 else None
    print(json.dumps({
        "metric": "emulator vs CPM cost per parameter point", "value": r["cost_ratio"], "unit": "x",
        "n_gpus": 1, "steps": args.emu_epochs, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "emulator-6-256-256-256-8", **{k: r[k] for k in ("n_train", "n_train_points",
                                                                               "train_reps", "n_test", "replicates",
                                                                               "plan", "L_range", "epochs")}},
        "emulator": r, "roofline": None, "cpu_baseline": cpu_fields(cpu)}), flush=True)


def emulator_cpu_baseline(args):
    """The same cost ratio with both sides on one pinned CPU thread: the
    oracle's CPM run per parameter point (a few MCS of sample points, scaled
    to the study's MCS per run) against the FP64 reference MLP's forward pass
    per point."""
    import numpy as np
    import oracle
    from oracle import mlp
    from paper_2312_09317_amd import emulator
    plan = emulator.RunPlan()
    pts = emulator.points(16, seed=1)
    n_mcs = sample_mcs(args, 100)

    def cpm_side():
        t = 0.0
        for q in pts:
            w = q.workload()
            st = oracle.State(oracle_model(w), w.lattice, w.cell_type, w.act)
            t0 = time.perf_counter()
            st.sweep(n_mcs)
            t += time.perf_counter() - t0
        return t / len(pts) * plan.n_mcs / n_mcs

    def mlp_side():
        W, b = mlp.init(0)
        x = np.random.default_rng(0).standard_normal((65536, 6))
        t0 = time.perf_counter()
        mlp.forward(W, b, x)
        return (time.perf_counter() - t0) / 65536
    (cpm_s, cpu_id) = pinned(cpm_side)
    (mlp_s, _) = pinned(mlp_side)
    return {"value": cpm_s / mlp_s, "unit": "x", "cores": 1, "kind": "oracle",
            "sample": f"oracle CPM: {len(pts)} parameter points x {n_mcs} MCS, scaled to {plan.n_mcs} MCS per run "
                      f"({cpm_s:.2f} s per point); FP64 reference MLP: 65,536 points ({mlp_s * 1e6:.2f} us per "
                      f"point); one thread pinned to CPU {cpu_id}",
            "host_cpus": host_cpus(), "pinned_cpu": cpu_id}


if __name__ == "__main__":
    main()
