"""Host-side logic of bench.py: algorithmic bytes per kernel group, the roofline record and
the one-GPU guard.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

WORK = {"tri_list_wave": 1000, "tri_list_wg": 2000, "triangles_wave": 10, "triangles_wg": 20,
        "wedges_wave": 100, "wedges_mid": 200, "wedges_wg": 300, "wedges_huge": 400}


def test_group_bytes_per_unit_figures():
    # per-edge, 4-byte credits, triangle records on
    gb = bench.group_bytes(WORK, per_edge=True, acc_bytes=4, records=True)
    assert gb["tri_wave"] == 4 * 1000 + (4 + 4 + 16) * 10
    assert gb["tri_wg"] == 4 * 2000 + (4 + 4 + 16) * 20
    assert gb["wedge_wave"] == 8 * 100 and gb["wedge_mid"] == 8 * 200
    assert gb["wedge_wg"] == 8 * 300 and gb["wedge_huge"] == 8 * 400
    assert gb["gather_wave"] == 8 * 10 + (12 + 8) * 10
    assert gb["gather_wg"] == 8 * 20 + (12 + 8) * 20
    # records off: the gather pass re-scans the lists
    gb = bench.group_bytes(WORK, per_edge=True, acc_bytes=8, records=False)
    assert gb["gather_wave"] == 4 * 1000 + (12 + 16) * 10
    assert gb["tri_wave"] == 4 * 1000 + (4 + 8) * 10
    # global counts only: no credits, no gather pass
    gb = bench.group_bytes(WORK, per_edge=False, acc_bytes=4, records=True)
    assert "gather_wave" not in gb and "gather_wg" not in gb
    assert gb["wedge_wg"] == 4 * 300
    assert gb["tri_wg"] == 4 * 2000 + (4 + 16) * 20


def test_roofline_takes_the_longest_group():
    timing = {"tri_wave": 1.0, "tri_wg": 0.5, "gather_wave": 0.1, "gather_wg": 0.1,
              "wedge_wave": 0.2, "wedge_mid": 0.3, "wedge_wg": 2.0, "wedge_huge": 0.0}
    r = bench.roofline(timing, WORK, per_edge=True, acc_bytes=4, workload="er_1k")
    assert r["group"] == "wedge_wg" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["alg_bytes"] == 8 * 300
    assert r["achieved"] == pytest.approx(8 * 300 / 2.0e-3 / 1e9, abs=0.05)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    assert r["peak"] == 8000.0
    assert r["traffic"] is None   # counters belong to another workload


def test_traffic_only_for_its_workload_and_mode():
    assert bench.measured_traffic("er_1k", True, "wedge_wg") is None
    assert bench.measured_traffic("chung_lu_1m", False, "wedge_wg") is None
    for wl, rec in bench.TRAFFIC["workloads"].items():
        v = bench.measured_traffic(wl, True, "wedge_wg")
        assert v is None or v == rec["wedge_wg"]


def test_prep_competes_and_atomic_roof():
    timing = {"tri_wave": 1.0, "tri_wg": 0.5, "gather_wave": 0.1, "gather_wg": 0.1,
              "wedge_wave": 0.2, "wedge_mid": 0.3, "wedge_wg": 2.0, "wedge_huge": 0.0, "prep": 3.0}
    pb = bench.prep_bytes(100, 1000, 8)
    assert pb == (8 * 1000 + 8 * 101) + (8 * 1000 + 4 * 101) + (4 * 1000 + 4 * 101)
    r = bench.roofline(timing, WORK, per_edge=True, acc_bytes=4, prep=pb,
                       atomic_rate={"rate": 1e9, "what": "test"})
    assert r["group"] == "prep" and r["alg_bytes"] == pb and "atomic_roof" not in r
    timing["prep"] = 0.1
    r = bench.roofline(timing, WORK, per_edge=True, acc_bytes=4, prep=pb,
                       atomic_rate={"rate": 1e9, "what": "test"})
    assert r["group"] == "wedge_wg"
    a = r["atomic_roof"]
    assert a["atomics"] == 300 and a["frac"] == pytest.approx(300 / 2.0e-3 / 1e9, abs=1e-4)
    assert r["closest_roof"] in ("hbm", "atomics")
    # global counts only: the wedge pass issues no per-wedge global atomics
    r = bench.roofline(timing, WORK, per_edge=False, acc_bytes=4, prep=pb,
                       atomic_rate={"rate": 1e9, "what": "test"})
    assert "atomic_roof" not in r


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr


def test_parse_schedule():
    assert bench.parse_schedule("wedge_stream=1, list_order=1") == {"wedge_stream": 1, "list_order": 1}
    assert bench.parse_schedule("") == {}
    assert bench.parse_schedule(None) == {}


def test_resolved_schedule():
    auto = {"wedge_stream": -1, "list_order": -1}
    assert bench.resolved_schedule(auto, 1 << 25) == {"wedge_stream": 2, "list_order": 1}
    assert bench.resolved_schedule(auto, (1 << 25) - 1) == {"wedge_stream": 2, "list_order": 2}
    assert bench.resolved_schedule(auto, 1 << 28, batch=True) == {"wedge_stream": 2, "list_order": 2}
    assert bench.resolved_schedule({"wedge_stream": 0, "list_order": 3}, 1 << 30) == {"wedge_stream": 0, "list_order": 3}


def test_side_run_settings():
    """The short batch run beside the R-MAT line sets a valid schedule; the served run a
    short stream over small pools."""
    sc = bench.parse_schedule(bench.SIDE_BATCH["schedule"])
    assert sc == {"wedge_wave_max": 128, "wedge_mid_max": 4096, "wedge_dense": 4096, "wedge_stream": 1}
    assert bench.SIDE_BATCH["steps"] >= 1 and bench.SIDE_SERVED["seconds"] <= 30
