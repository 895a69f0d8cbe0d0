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


def test_traffic_records_match_their_kernel_source():
    # stored HBM traffic is reported only for the kernel source it was
    # measured on; each record names its commands and calibration factors
    import glob
    sys.path.insert(0, ROOT)
    import bench
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")):
        with open(path) as fh:
            rec = json.load(fh)
        assert rec["kernel"] in bench.ROCPROF_NAME and rec["workload"] in bench.WORKLOADS
        assert all(c.startswith("rocprofv3 --pmc ") for c in rec["commands"])
        assert 0 < rec["fetch_factor"] and 0 < rec["write_factor"]
        assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
        got = bench.measured_traffic(rec["kernel"], rec["workload"])
        assert got is None or got == rec["hbm_bytes_per_launch"]


def test_write_traffic_scales_by_the_copy_dispatch(tmp_path, monkeypatch):
    # two synthetic counter files: the kernel reads 3 GiB and writes 1 GiB per
    # launch while the counters read half of what the 1 GiB copy moves on
    # fetch and all of it on write
    sys.path.insert(0, ROOT)
    import bench
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    kib = 1 << 20
    name = "void tnb::medf_bin_pipe<0, 1, 0, double>(tnb::MedF, double const*)"
    fetch = hdr + "".join("%d,%s,FETCH_SIZE,%r\n" % (d, '"%s"' % name, 1.5 * kib) for d in (1, 2)) \
        + "3,__amd_rocclr_copyBuffer,FETCH_SIZE,%r\n" % (0.5 * kib)
    write = hdr + "".join("%d,%s,WRITE_SIZE,%r\n" % (d, '"%s"' % name, 1.0 * kib) for d in (1, 2)) \
        + "3,__amd_rocclr_copyBuffer,WRITE_SIZE,%r\n" % (1.0 * kib)
    (tmp_path / "f.csv").write_text(fetch)
    (tmp_path / "w.csv").write_text(write)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "medf_Y2", "zephyr_z2_t4_plain")
    rec = json.loads((tmp_path / "profiles" / "medf_Y2_zephyr_z2_t4_plain_traffic.json").read_text())
    assert rec["launches"] == 2
    assert rec["fetch_bytes_per_launch"] == 3 * (1 << 30) and rec["write_bytes_per_launch"] == 1 << 30
