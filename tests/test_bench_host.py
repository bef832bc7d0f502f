"""Host-side checks of bench.py (no GPU): the one-GPU contract and the consistency of the
committed counter records with the kernel sources they were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_counter_records_match_the_kernel_sources():
    """Every product of both paths has a counter record, taken on the kernel sources as they
    stand (bench.py reports traffic and the MFMA busy fraction only then), with the
    calibration scales and a summary file that exists."""
    recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key in ("w_mnij_mixed", "w_mbej_mixed", "ring_mixed", "pp_ladder_mixed",
                "w_mnij_fp64", "w_mbej_fp64", "ring_fp64", "pp_ladder_fp64", "hh_ladder_fp64"):
        rec = bench.measured_record(key)
        assert rec is not None, key
        assert rec["hbm_bytes_per_launch"] > 0 and 0.0 < rec["mfma_busy"] < 1.0 and 1.0 < rec["clock_ghz"] < 2.5
        assert os.path.exists(os.path.join(ROOT, rec["summary"]))
        assert recs[key]["fetch_scale"] == 2.0 and 0.9 <= recs[key]["write_scale"] <= 1.0
