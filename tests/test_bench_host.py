"""Host logic of bench.py on the CPU: the one-GPU refusal and the gating of
measured HBM traffic by the kernel sources' hash and the layout."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _table(sha, layout="in_place"):
    return {"sources_sha256": sha, "layout": layout, "fetch_kib": 100.0, "write_kib": 10.0,
            "fetch_scale": 2.0, "write_scale": 1.0}


def test_traffic_scales_the_counters():
    t = _table(bench.kernel_sources_sha())
    assert bench.measured_traffic_bytes("in_place", t) == (2.0 * 100.0 + 10.0) * 1024.0
    assert bench.measured_traffic_bytes(None, t) == (2.0 * 100.0 + 10.0) * 1024.0


def test_traffic_is_withheld_for_other_sources_or_layouts():
    cur = bench.kernel_sources_sha()
    other = "0" * 16 if cur != "0" * 16 else "1" * 16
    assert bench.measured_traffic_bytes("in_place", _table(other)) is None
    assert bench.measured_traffic_bytes("box", _table(cur)) is None


def test_tables_are_well_formed():
    for t in (bench.MEASURED_TRAFFIC, bench.MEASURED_TRAFFIC_TISSUE, bench.MEASURED_TRAFFIC_SORTING,
              bench.MEASURED_TRAFFIC_COLLECTIVE, bench.MEASURED_TRAFFIC_BATCH):
        assert len(t["sources_sha256"]) == 16
        assert t["fetch_kib"] > 0 and t["write_kib"] > 0
        assert (t["fetch_scale"], t["write_scale"]) == (2.0, 1.0)


def test_traffic_is_keyed_on_the_tile():
    t = dict(_table(bench.kernel_sources_sha()), tile=[64, 2, 2])
    assert bench.measured_traffic_bytes("in_place", t, tile=(64, 2, 2)) is not None
    assert bench.measured_traffic_bytes("in_place", t, tile=(64, 4, 1)) is None


def test_roofline_reports_both_fractions():
    r = bench.roofline_fields(4000.0, 40e6, 10e-6, "k", 256.0)
    assert r["frac"] == 0.5 and r["peak"] == 8000.0
    assert abs(r["achieved_measured_bytes"] - 4000.0) < 1e-9 and abs(r["frac_measured_bytes"] - 0.5) < 1e-12
    r = bench.roofline_fields(4000.0, None, 10e-6, "k", 256.0)
    assert r["traffic"] is None and r["frac_measured_bytes"] is None


def test_pinned_restores_the_affinity():
    before = os.sched_getaffinity(0)
    out, cpu = bench.pinned(lambda: os.sched_getaffinity(0))
    assert out == {cpu} and cpu in before
    assert os.sched_getaffinity(0) == before
