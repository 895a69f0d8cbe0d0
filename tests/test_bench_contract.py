"""bench.py's command-line contract that can be checked without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_traffic_record_matches_its_kernel_source():
    # the stored HBM traffic is reported only for the kernel source it was
    # measured on; the record must name its command and calibration
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert rec["kernel"] == "medf_Y2" and rec["workload"] in bench.WORKLOADS
    assert all(c.startswith("rocprofv3 --pmc ") for c in rec["commands"])
    cal = rec["copy_calibration"]
    assert abs(cal["fetch_kib"] / (cal["bytes"] / 1024) - cal["fetch_factor"]) < 1e-9
    assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    got = bench.measured_traffic("medf_Y2", rec["workload"])
    assert got is None or got == rec["hbm_bytes_per_launch"]
