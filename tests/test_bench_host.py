"""Host-side checks of the benchmark's bookkeeping (no GPU needed).

  * the roofline takes the launched kernel with the most device time, divides
    its algorithmic flops per launch by the mean HIP-event launch time and
    the published 157.3 TFLOP/s, and scales per-workgroup traffic by the
    blocks of a launch; a resident (persistent) record, when there is one,
    is the dominant kernel instead;
  * the device-side entry rate ignores resident records;
  * the CPU-only oracle H-matrix leg runs the oracle's partition and ACA on a
    sample of blocks and extrapolates by summed block dimensions;
  * more than one GPU is refused with a message.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1711_01897_amd import inputs  # noqa: E402


def _rec(op=0, space=1, prec=1, q=6, persistent=0, launches=10, workgroups=5000, blocks=5000, entries=1000000,
         evals=4.0e8, seconds=2.0e-4, seconds_events=2.5e-4):
    return {"op": op, "space": space, "prec": prec, "quad_points": q, "persistent": persistent,
            "launches": launches, "workgroups": workgroups, "blocks": blocks, "entries": entries,
            "pair_evals": evals, "triangle_loads": 0, "seconds": seconds, "seconds_events": seconds_events}


def test_roofline_of_the_launched_kernel():
    small = _rec(op=1, seconds=1e-5, seconds_events=1e-5)
    big = _rec()
    roof, dom = bench.roofline([small, big], workload="no_such_workload")
    assert dom is big and roof["kernel"] == "k_p1_f32<op=0,Q=6>" and not roof["persistent"]
    per_launch = 4.0e8 * bench.FLOPS_PER_EVAL[(0, 1)] / 10
    achieved = per_launch / 2.5e-5
    assert roof["achieved"] == pytest.approx(achieved / 1e12, abs=1e-3)
    assert roof["frac"] == pytest.approx(achieved / 157.3e12, abs=1e-4)
    assert roof["peak"] == 157.3 and roof["traffic"] is None
    assert roof["mean_launch_us"] == pytest.approx(25.0) and roof["blocks_per_launch"] == 500
    assert roof["algorithmic_bytes_per_launch"] == pytest.approx(80.0 * 1e6 / 10)


def test_roofline_prefers_resident_launches_and_scales_traffic_by_blocks(tmp_path, monkeypatch):
    launched = _rec(seconds=9.0)
    resident = _rec(persistent=1, launches=2, workgroups=2 * 769, blocks=40000, seconds=1.0, seconds_events=1.0)
    rec = tmp_path / "traffic.json"
    rec.write_text('{"kernel_source_hash": "%s", "bytes_per_workgroup": 1000.0}' % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "traffic_file", lambda workload: str(rec))
    roof, dom = bench.roofline([launched, resident])
    assert dom is resident and roof["persistent"] and roof["kernel"] == "kp_p1_f32<op=0,Q=6>"
    assert roof["blocks_per_launch"] == 20000 and roof["traffic"] == pytest.approx(1000.0 * 20000)
    # a record taken with another kernel source is not used
    rec.write_text('{"kernel_source_hash": "0000", "bytes_per_workgroup": 1000.0}')
    assert bench.roofline([launched])[0]["traffic"] is None


def test_kernel_entry_rate_ignores_resident_records():
    a = _rec(entries=3000, seconds=2.0, seconds_events=3.0)
    b = _rec(entries=10, seconds=1.0, seconds_events=1.0)
    r = _rec(persistent=1, seconds=100.0)
    assert bench.kernel_entries_rate([a, b, r]) == pytest.approx(1000.0)
    assert bench.kernel_entries_rate([r]) is None


def test_cpu_hmatrix_leg_on_a_small_sphere():
    xyz, tri = inputs.icosphere(4)
    out = bench.cpu_hmatrix(inputs, xyz, tri, [0], 0.05)
    assert out["kind"] == "oracle" and out["admissible_blocks"] > 0
    assert 1 <= out["sampled_blocks"] <= out["admissible_blocks"]
    single = out["ops"]["single"]
    assert single["sampled_entries"] > 0 and single["mean_rank"] >= 1
    assert single["extrapolated_seconds_all_admissible_blocks"] >= single["sampled_seconds"]
    assert out["extrapolated_seconds"] == pytest.approx(single["extrapolated_seconds_all_admissible_blocks"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert "one GPU" in (r.stdout + r.stderr)
