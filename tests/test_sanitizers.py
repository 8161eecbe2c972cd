"""Host code under the sanitizers (CPU only).

Three programs in tests/sanitize/ are built and run here:
  - oracle_asan: the CPU oracle (oracle/mg_oracle.c) under AddressSanitizer
    and UndefinedBehaviorSanitizer, on exact-size heap operands.
  - abi_asan: the C ABI's validation and host-side helpers (every entry
    point's argument errors, layout queries, work-division and tuning
    rules, batch validation, the server's request checks) under ASan+UBSan,
    against a libmg whose host code is instrumented.
  - server_tsan: the serving loop's scheduler, completion waiters and replay
    submitter under ThreadSanitizer, in host-simulation mode, with several
    threads submitting, polling, waiting and reading statistics at once.
The library is compiled as usual for gfx950 with the sanitizer applied to the
host compilation only (nothing here launches a kernel); the drivers are
plain C++ against include/mg.h.
Each program must exit 0 and its output must hold no sanitizer report.
"""

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1602_08477_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/lib/llvm/bin/clang++"  # the drivers are plain C++ against mg.h
REPORTS = ("ERROR: AddressSanitizer", "WARNING: ThreadSanitizer", "runtime error:",
           "ERROR: LeakSanitizer")

pytestmark = pytest.mark.skipif(not (shutil.which("gcc") and os.path.exists(HIPCC)),
                                reason="needs gcc and hipcc")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    return r.returncode, r.stdout, err


def _host_lib(tag, san):
    """libmg with instrumented host code."""
    d = os.path.join(OUT, tag)
    os.makedirs(d, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g",
             "-fno-omit-frame-pointer", "-std=c++17", "-fPIC", "-Xarch_host",
             f"-fsanitize={san}", "-I" + os.path.join(ROOT, "include")]

    def one(src):
        obj = os.path.join(d, os.path.basename(src) + ".o")
        rc, _, err = _run([HIPCC, *flags, "-c", src, "-o", obj])
        assert rc == 0, f"{src}:\n{err}"
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(one, srcs))
    lib = os.path.join(d, "libmg_san.so")
    rc, _, err = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-Xarch_host",
                       f"-fsanitize={san}", "-o", lib, *objs, "-lpthread"])
    assert rc == 0, err
    return d


def _program(tag, san, driver):
    d = _host_lib(tag, san)
    exe = os.path.join(d, os.path.splitext(os.path.basename(driver))[0])
    rc, _, err = _run([CLANGXX, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
                       f"-fsanitize={san}", "-I" + os.path.join(ROOT, "include"), driver,
                       "-o", exe, "-L" + d, "-lmg_san", "-Wl,-rpath," + d, "-lpthread"])
    assert rc == 0, err
    return exe


def _check(rc, out, err):
    text = out + err
    assert rc == 0, text[-4000:]
    for rep in REPORTS:
        assert rep not in text, text[-4000:]


def test_oracle_under_asan_ubsan():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_asan")
    rc, _, err = _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                       "-mfma", "-fopenmp", "-std=c11", "-fsanitize=address,undefined",
                       "-fno-sanitize-recover=undefined",
                       os.path.join(HERE, "oracle_asan.c"),
                       os.path.join(ROOT, "oracle", "mg_oracle.c"), "-o", exe, "-lm"])
    assert rc == 0, err
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, out, err = _run([exe], env=env)
    _check(rc, out, err)
    assert "0 failures" in out


def test_c_abi_validation_under_asan_ubsan():
    exe = _program("asan", "address,undefined", os.path.join(HERE, "abi_asan.cpp"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, out, err = _run([exe], env=env)
    _check(rc, out, err)
    assert "0 failures" in out


def test_server_threads_under_tsan():
    exe = _program("tsan", "thread", os.path.join(HERE, "server_tsan.cpp"))
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    rc, out, err = _run([exe], env=env)
    _check(rc, out, err)
    assert "0 failures" in out
