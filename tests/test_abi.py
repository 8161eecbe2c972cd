"""The C-ABI library loads, exports every declared symbol and rejects bad
arguments before enqueuing anything (no GPU needed: these paths make no HIP
calls)."""

import ctypes
import os
import re

import pytest

import paper_1602_08477_amd as mg
from helpers import NAIVE_CFG, NATIVE_CFGS, SPLIT_CFGS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]

FAKE = ctypes.c_void_p(0x10000000)  # never dereferenced: validation fails first
FAKE_B = ctypes.c_void_p(0x20000000)
FAKE_C = ctypes.c_void_p(0x30000000)
NULL = ctypes.c_void_p(0)


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(mg_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 10
    L = mg.lib()
    for n in names:
        assert hasattr(L, n), n


def test_version_and_cfgs():
    assert mg.lib().mg_version() >= 10000
    assert mg.num_tile_cfgs() == NATIVE_CFGS  # the GPU parity tests cover every one of them
    for c in range(mg.num_tile_cfgs()):
        info = mg.tile_cfg_info(c)
        if c == NAIVE_CFG:
            assert info == {"bm": 16, "bn": 16, "bk": 1, "threads": 256}
            assert mg.tile_cfg_info(c, mg.F32) == info
            continue
        assert info["bm"] % 32 == 0 and info["bn"] % 32 == 0 and info["threads"] in (256, 512, 1024)
        assert mg.tile_cfg_info(c, mg.F32)["bk"] == 2 * info["bk"]
    assert mg.NAIVE_CFG == NAIVE_CFG
    with pytest.raises(mg.MgError):
        mg.tile_cfg_info(99)
    assert mg.pick_tile_cfg(8192, 8192, 8192) == 21
    assert mg.pick_tile_cfg(2048, 2048, 2048) == 23
    assert mg.pick_tile_cfg(2048, 2048, 2048, mg.F32) == 21
    assert mg.pick_tile_cfg(4096, 4096, 4096) == 21
    assert mg.pick_tile_cfg(8192, 1024, 4096) == 21
    assert mg.pick_tile_cfg(1024, 8192, 8192) == 21
    assert mg.pick_tile_cfg(1024, 1024, 1024) == 26
    assert mg.pick_tile_cfg(1536, 1536, 1536) == 29
    assert mg.pick_tile_cfg(1024, 1024, 1024, mg.F32) == 26
    assert mg.pick_tile_cfg(512, 512, 512) == 19
    assert mg.pick_tile_cfg(4096, 4096, 4096, mg.F32) == 22
    assert 0 <= mg.pick_tile_cfg(16, 16, 16) < mg.num_tile_cfgs()


def call_gemm(dt=mg.F64, algo=mg.NATIVE, m=8, n=8, k=8, A=FAKE, lda=8, B=FAKE_B, ldb=8,
              C=FAKE_C, ldc=8, alpha=1.0, beta=0.0):
    return mg.lib().mg_gemm(dt, algo, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, NULL)


@pytest.mark.parametrize("kw,code", [
    (dict(m=-1), mg.ERR_INVALID_ARG),
    (dict(k=-3), mg.ERR_INVALID_ARG),
    (dict(A=NULL), mg.ERR_INVALID_ARG),
    (dict(B=NULL), mg.ERR_INVALID_ARG),
    (dict(C=NULL), mg.ERR_INVALID_ARG),
    (dict(lda=7), mg.ERR_INVALID_ARG),
    (dict(ldb=7), mg.ERR_INVALID_ARG),
    (dict(ldc=7), mg.ERR_INVALID_ARG),
    (dict(dt=7), mg.ERR_INVALID_ARG),
    (dict(algo=9), mg.ERR_INVALID_ARG),
    (dict(dt=mg.F32, algo=mg.SPLIT_I8), mg.ERR_UNSUPPORTED),
    (dict(C=FAKE), mg.ERR_INVALID_ARG),               # C overlaps A
    (dict(C=ctypes.c_void_p(0x20000100)), mg.ERR_INVALID_ARG),  # C overlaps B
    (dict(A=ctypes.c_void_p(0x10000004)), mg.ERR_INVALID_ARG),  # misaligned double
    (dict(m=1 << 31), mg.ERR_INVALID_ARG),
])
def test_invalid_arguments(kw, code):
    assert call_gemm(**kw) == code
    assert mg.last_error() != ""


def test_problems_array_passes_through():
    probs = [mg.Problem(8, 8, 8, 1.0, 0.0, 0x1000 * i, 8, 0x1000 * i + 512, 8,
                        0x1000 * i + 1024, 8) for i in range(5)]
    arr = mg.problems_array(probs)
    assert mg._problems(arr) is arr and arr[1] == 5
    built, n = mg._problems(probs)
    assert n == 5 and [built[i].A for i in range(5)] == [p.A for p in probs]


def test_release_build_flags():
    assert mg.build_flags() == 0


def _fake_batch(count):
    P = mg.Problem * count
    return P(*[mg.Problem(8, 8, 8, 1.0, 1.0, 0x10000000 + 0x1000 * (3 * i), 8,
                          0x10000000 + 0x1000 * (3 * i + 1), 8,
                          0x10000000 + 0x1000 * (3 * i + 2), 8) for i in range(count)])


def test_batched_algorithm_checks_without_gpu():
    """mg_gemm_batched: split algorithms take FP64 only, unknown algorithms
    and bad descriptors are rejected before anything touches a device."""
    arr = _fake_batch(3)
    assert mg.lib().mg_gemm_batched(mg.F32, mg.SPLIT_I8, 3, arr, NULL) == mg.ERR_UNSUPPORTED
    assert mg.lib().mg_gemm_batched(mg.F32, mg.SPLIT_BF16, 3, arr, NULL) == mg.ERR_UNSUPPORTED
    assert mg.lib().mg_gemm_batched(mg.F64, 9, 3, arr, NULL) == mg.ERR_INVALID_ARG
    arr[1].lda = 2
    for algo in (mg.SPLIT_I8, mg.SPLIT_BF16):
        assert mg.lib().mg_gemm_batched(mg.F64, algo, 3, arr, NULL) == mg.ERR_INVALID_ARG
        assert "problem 1" in mg.last_error()
    arr[1].lda = 8
    arr[2].C = arr[0].C  # outputs overlap
    assert mg.lib().mg_gemm_batched(mg.F64, mg.SPLIT_I8, 3, arr, NULL) == mg.ERR_INVALID_ARG
    assert mg.lib().mg_gemm_batched(mg.F64, mg.SPLIT_I8, 0, None, NULL) == mg.OK


def test_empty_problem_is_ok_without_gpu():
    assert call_gemm(m=0) == mg.OK
    assert call_gemm(n=0, C=NULL) == mg.OK
    assert mg.last_error() == ""


def test_alpha_zero_allows_null_ab():
    # alpha == 0: A and B are not read, so NULL passes validation; the call
    # would then enqueue C <- beta*C, so only the validator is exercised here
    L = mg.lib()
    assert L.mg_gemm_cfg(mg.F64, 99, 8, 8, 8, 0.0, NULL, 8, NULL, 8, 1.0, FAKE_C, 8, NULL) \
        == mg.ERR_INVALID_ARG
    assert "cfg" in mg.last_error()


def test_split_layout_and_errors():
    L = mg.split_layout(mg.SPLIT_I8, 7, 100, 300, 300)
    assert (L["mp"], L["np"], L["kp"], L["elem_bytes"]) == (256, 512, 384, 1)
    assert L["a_off"] % 256 == 0 and L["b_off"] % 256 == 0
    assert L["b_off"] >= L["a_off"] + 7 * 256 * 384
    assert L["p_off"] >= L["b_off"] + 7 * 512 * 384
    assert L["total_bytes"] >= L["p_off"] + 8 * 256 * 512
    Lb = mg.split_layout(mg.SPLIT_BF16, 6, 1, 1, 1)
    assert (Lb["mp"], Lb["np"], Lb["kp"], Lb["elem_bytes"]) == (256, 256, 128, 2)
    assert mg.split_num_cfgs() == SPLIT_CFGS
    assert mg.split_default_slices(mg.SPLIT_I8) == 7
    assert mg.split_default_slices(mg.SPLIT_BF16) == 6
    with pytest.raises(mg.MgError):
        mg.split_layout(mg.SPLIT_I8, 0, 4, 4, 4)
    with pytest.raises(mg.MgError):
        mg.split_layout(mg.SPLIT_I8, 17, 4, 4, 4)
    with pytest.raises(mg.MgError):
        mg.split_layout(mg.NATIVE, 7, 4, 4, 4)
    lib = mg.lib()
    # workspace too small
    rc = lib.mg_gemm_split(mg.SPLIT_I8, 7, 8, 8, 8, 1.0, FAKE, 8, FAKE_B, 8, 0.0, FAKE_C, 8,
                           ctypes.c_void_p(0x40000000), 16, NULL)
    assert rc == mg.ERR_INVALID_ARG and "workspace" in mg.last_error()
    # workspace overlapping C
    rc = lib.mg_gemm_split(mg.SPLIT_I8, 7, 8, 8, 8, 1.0, FAKE, 8, FAKE_B, 8, 0.0, FAKE_C, 8,
                           FAKE_C, 1 << 20, NULL)
    assert rc == mg.ERR_INVALID_ARG


def call_gemm_ex(dt=mg.F64, cfg=-1, ta=0, tb=0, m=8, n=6, k=4, A=FAKE, lda=None, B=FAKE_B,
                 ldb=None, C=FAKE_C, ldc=6, alpha=1.0, beta=0.0):
    lda = (m if ta else k) if lda is None else lda
    ldb = (k if tb else n) if ldb is None else ldb
    return mg.lib().mg_gemm_ex(dt, cfg, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                               NULL)


@pytest.mark.parametrize("kw,code,needle", [
    (dict(ta=2), mg.ERR_INVALID_ARG, "trans"),
    (dict(tb=-1), mg.ERR_INVALID_ARG, "trans"),
    (dict(cfg=-2), mg.ERR_INVALID_ARG, "cfg"),
    (dict(cfg=NATIVE_CFGS), mg.ERR_INVALID_ARG, "cfg"),
    (dict(dt=5), mg.ERR_INVALID_ARG, "dtype"),
    # stored A^T is k x m: its pitch must cover m, not k
    (dict(ta=1, lda=4), mg.ERR_INVALID_ARG, "lda"),
    (dict(ta=0, lda=3), mg.ERR_INVALID_ARG, "lda"),
    # stored B^T is n x k: its pitch must cover k, not n
    (dict(tb=1, ldb=3), mg.ERR_INVALID_ARG, "ldb"),
    (dict(tb=0, ldb=5), mg.ERR_INVALID_ARG, "ldb"),
    # C placed inside the stored extent of A^T (k rows of pitch m: 32 doubles)
    (dict(ta=1, C=ctypes.c_void_p(0x10000000 + 8 * 30)), mg.ERR_INVALID_ARG, "overlap"),
    # C inside the stored extent of B^T (n rows of pitch k: 24 doubles)
    (dict(tb=1, C=ctypes.c_void_p(0x20000000 + 8 * 20)), mg.ERR_INVALID_ARG, "overlap"),
    (dict(ta=1, A=NULL), mg.ERR_INVALID_ARG, "NULL"),
])
def test_gemm_ex_invalid_arguments(kw, code, needle):
    assert call_gemm_ex(**kw) == code
    assert needle in mg.last_error()


def test_gemm_ex_empty_problem_is_ok_without_gpu():
    assert call_gemm_ex(m=0, ta=1, lda=1) == mg.OK
    assert call_gemm_ex(n=0, tb=1, C=NULL) == mg.OK
    assert mg.last_error() == ""


def call_daxpy(n=8, alpha=1.0, x=FAKE, incx=1, y=FAKE_B, incy=1):
    return mg.lib().mg_daxpy(n, alpha, x, incx, y, incy, NULL)


@pytest.mark.parametrize("kw,needle", [
    (dict(n=-1), "negative"),
    (dict(incx=0), "increments"),
    (dict(incy=-2), "increments"),
    (dict(x=NULL), "NULL"),
    (dict(y=NULL), "NULL"),
    (dict(x=ctypes.c_void_p(0x10000004)), "aligned"),
    (dict(y=ctypes.c_void_p(0x10000000 + 8 * 7)), "overlap"),        # inside x
    (dict(y=FAKE, incy=2), "overlap"),                               # x itself, other increment
    (dict(n=1 << 62), "overflow"),
])
def test_daxpy_invalid_arguments(kw, needle):
    assert call_daxpy(**kw) == mg.ERR_INVALID_ARG
    assert needle in mg.last_error()


def test_daxpy_quick_returns_without_gpu():
    assert call_daxpy(n=0, x=NULL, y=NULL) == mg.OK
    assert call_daxpy(alpha=0.0, x=NULL, y=NULL) == mg.OK
    assert mg.last_error() == ""
