"""The library-overhead driver (drivers/overhead.hip) runs and reports every
shape (needs a GPU).  Its numbers are measurements, not pass/fail bars; the
naive work division's results are checked by the parity tests of every cfg."""

import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

mg = pytest.importorskip("paper_1602_08477_amd")


def test_overhead_driver_reports_all_shapes():
    from paper_1602_08477_amd import build as b
    exe = b.driver_path(os.path.join(b.HERE, "drivers", "overhead.hip"))
    assert os.path.exists(exe), "build first"
    r = subprocess.run([exe, "5"], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert [s["n"] for s in rec["shapes"]] == [64, 256, 1024, 2048, 4096]
    for s in rec["shapes"]:
        assert s["device_ms_mg_gemm"] > 0 and s["device_ms_direct"] > 0 and s["naive_ms"] > 0
