"""Host logic of bench.py (CPU only): the one-GPU rule, the counter ingest
with its copy calibration, the traffic record's kernel-source check, and the
roofline arithmetic."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _counter_csv(path, counter, fwd_kib, copy_kib, n_fwd=3):
    fields = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for _ in range(n_fwd):
            w.writerow({"Kernel_Name": "void (anonymous namespace)::k_forward<false, 0, true, false>(FwdArgs)",
                        "Grid_Size": 524288, "Counter_Name": counter, "Counter_Value": fwd_kib})
        for _ in range(3):
            w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 1 << 20, "Counter_Name": counter,
                        "Counter_Value": copy_kib})


def test_ingest_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    out = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "PROFILE_COUNTERS", str(out))
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    copy_kib = bench.CALIB_COPY_BYTES / 1024
    _counter_csv(f, "FETCH_SIZE", 1000.0, copy_kib / 2)     # counter reads half of the copy
    _counter_csv(w, "WRITE_SIZE", 3000.0, copy_kib)
    bench.ingest_counters(str(f), str(w))
    rec = json.loads(out.read_text())
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == 2000 * 1024 and rec["write_bytes_per_launch"] == 3000 * 1024
    assert rec["kernel_source_sha"] == bench.kernel_source_sha()
    tr = bench.traffic_from_profile(str(out))
    assert tr["fetch_bytes"] + tr["write_bytes"] == 5000 * 1024
    rec["kernel_source_sha"] = "0" * 16                      # counters of another kernel are not reported
    out.write_text(json.dumps(rec))
    assert bench.traffic_from_profile(str(out)) is None


def test_roofline_arithmetic():
    r = bench.rooflines(n_seg=1000, n_cross=400, n_node=7000, n_tri=1500, width=4, kern_ms=3.7e-5, traffic=None)
    ops = 15 * 4 * 7000 + 45 * 1500 + 250 * 1000
    assert r["alg_ops_per_launch"] == ops
    assert r["achieved"] == pytest.approx(ops / 3.7e-8 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.ALU_PEAK_TOPS, rel=1e-3)
    assert r["hbm_model"]["alg_bytes_per_launch"] == 112 * 7000 + 40 * 1500 + 8 * 400
    assert r["bound"] == "alu" and r["traffic"] is None
