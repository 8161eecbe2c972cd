"""LDS race check: every staged kernel, built with MG_LDS_POISON (each LDS
stage filled with 0xFF bytes before it is refilled), must give the release
build's results bit for bit.  A kernel that read a stage before its loads
had landed, or read bytes no load writes, would see NaN (FP) or -1 (INT8)
there and change its output.  The debug build runs in a child process
(MG_LIBRARY selects libmg_poison.so); the cases are in lds_poison_cases.py.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

from helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")

HERE = os.path.dirname(os.path.abspath(__file__))
POISON_LIB = os.path.join(os.path.dirname(mg.__file__), "libmg_poison.so")


def test_poisoned_lds_stages_change_nothing(tmp_path):
    if not os.path.exists(POISON_LIB):
        pytest.fail(f"{POISON_LIB} is missing: build() makes it next to libmg.so")
    import lds_poison_cases
    ref_path = str(tmp_path / "release.npz")
    got_path = str(tmp_path / "poison.npz")
    n = lds_poison_cases.run(ref_path)
    env = dict(os.environ, MG_LIBRARY=POISON_LIB)
    r = subprocess.run([sys.executable, os.path.join(HERE, "lds_poison_cases.py"), got_path],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    ref, got = np.load(ref_path), np.load(got_path)
    assert int(ref["build_flags"][0]) == 0, "parent must run the release build"
    assert int(got["build_flags"][0]) == mg.BUILD_LDS_POISON, "child did not load the debug build"
    assert sorted(ref.files) == sorted(got.files)
    bad = [name for name in ref.files if name != "build_flags" and
           not np.array_equal(ref[name], got[name], equal_nan=True)]
    nan = [name for name in ref.files if np.isnan(ref[name]).any()]
    log(f"lds poison: {n} outputs compared, {len(bad)} differ, {len(nan)} hold NaN")
    assert not nan, nan
    assert not bad, bad
