"""bench.py's contract on the CPU: one GPU only, and the committed HBM-traffic
records are internally consistent (no GPU needed)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_traffic_records_are_consistent():
    for name in ("traffic_dgemm_f64_n8192.json", "traffic_daxpy_n2p27.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
        cal = t["copy_calibration"]
        # the calibration copy reads and writes exactly its size
        assert abs(cal["fetch_kib_raw"] * cal["fetch_scale"] * 1024 - cal["bytes"]) < 1e-3 * cal["bytes"]
        assert abs(cal["write_kib_raw"] * cal["write_scale"] * 1024 - cal["bytes"]) < 1e-3 * cal["bytes"]
        fb = t["fetch_kib_per_launch_raw"] * cal["fetch_scale"] * 1024
        wb = t["write_kib_per_launch_raw"] * cal["write_scale"] * 1024
        assert abs(fb - t["fetch_bytes_per_launch"]) < 1e-4 * fb
        assert abs(wb - t["write_bytes_per_launch"]) < 1e-4 * wb
        assert t["bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
        assert t["bytes_per_launch"] >= 0.99 * t["algorithmic_bytes_per_launch"]
        assert len(t["kernel_source_hash"]) == 16
