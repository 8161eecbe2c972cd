"""Parity of the native FP64/FP32 HIP GEMM with the CPU oracle (needs a GPU).

Bars: FP64 relative Frobenius error <= 1e-13 against the compensated oracle
and, per element, the worst-case rounding bound (k+2)u(|alpha||A||B| +
|beta||C|); bit-exact results where every intermediate is exact (small
integers, identity); FP32 <= 1e-5 against the oracle run on the FP32-rounded
inputs.  Shapes span several tiles and ragged tails for every work division.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import (DMA_CFGS, KGROUP_CFGS, NATIVE_CFGS, elementwise_bound, host_mats, log,
                     to_dev, U32)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")

SHAPES = [(1, 1, 1), (7, 5, 3), (16, 16, 4), (33, 17, 65), (129, 130, 131), (64, 256, 31),
          (300, 200, 517), (256, 256, 256)]


def run(A, B, C, alpha, beta, cfg=None, dtype=torch.float64, lds=(None, None, None)):
    dA = None if A is None else to_dev(A, dtype, lds[0])
    dB = None if B is None else to_dev(B, dtype, lds[1])
    dC = to_dev(C, dtype, lds[2])
    mg.gemm(dA, dB, dC, alpha, beta, cfg=cfg, k=0 if A is None else None)
    torch.cuda.synchronize()
    return dC


def check_f64(got, A, B, C, alpha, beta, tag):
    ref = oracle.dgemm(alpha, A, B, beta, C)
    err = oracle.rel_fro_err(got, ref)
    bound = elementwise_bound(alpha, A, B, beta, C, A.shape[1])
    worst = float(np.max(np.abs(got - ref) / bound))
    log(f"{tag}: rel_fro_err={err:.3e} worst/bound={worst:.3f}")
    assert err <= 1e-13, (tag, err)
    assert worst <= 1.0, (tag, worst)


@pytest.mark.parametrize("cfg", range(NATIVE_CFGS))
@pytest.mark.parametrize("shape", SHAPES)
def test_native_f64_parity_all_cfgs(cfg, shape):
    m, n, k = shape
    log(f"native f64 cfg={cfg} shape={shape}")
    A, B, C = host_mats(synth.config_seed(1, 7) + m + 3 * n + 7 * k, m, n, k)
    got = run(A, B, C, 1.5, 0.5, cfg=cfg).cpu().numpy()
    check_f64(got, A, B, C, 1.5, 0.5, f"cfg{cfg} {shape}")


def test_native_f64_config1_n512():
    """Workload 1: n=512, U[-1,1), alpha=1.5, beta=0.5, default work division."""
    n = 512
    A, B, C = host_mats(synth.config_seed(1), n, n, n)
    got = run(A, B, C, 1.5, 0.5).cpu().numpy()
    check_f64(got, A, B, C, 1.5, 0.5, "config1 n=512")


@pytest.mark.parametrize("cfg", range(NATIVE_CFGS))
def test_small_integers_bit_exact(cfg):
    m, n, k = 150, 97, 301
    A = synth.small_int_matrix(31, 0, m, k)
    B = synth.small_int_matrix(31, 1, k, n)
    C = synth.small_int_matrix(31, 2, m, n)
    got = run(A, B, C, 1.5, 0.5, cfg=cfg).cpu().numpy()
    assert np.array_equal(got, 1.5 * (A @ B) + 0.5 * C)


def test_identity_and_diagonal_closed_forms():
    n = 200
    B = synth.matrix(32, 1, n, n)
    got = run(np.eye(n), B, np.zeros((n, n)), 1.0, 0.0).cpu().numpy()
    assert np.array_equal(got, B)
    d1 = synth.uniform_pm1(32, 3, n)
    d2 = synth.uniform_pm1(32, 4, n)
    C0 = synth.matrix(32, 2, n, n)
    got = run(np.diag(d1), np.diag(d2), C0, 1.0, 0.5).cpu().numpy()
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(got[off], (0.5 * C0)[off])
    assert np.array_equal(np.diag(got), d1 * d2 + 0.5 * np.diag(C0))


def test_rank_one_exact():
    m, k, n = 70, 90, 110
    u = synth.small_int_matrix(33, 0, m, 1)
    v = synth.small_int_matrix(33, 1, k, 1)
    w = synth.small_int_matrix(33, 2, k, 1)
    z = synth.small_int_matrix(33, 3, n, 1)
    got = run(u @ v.T, w @ z.T, np.zeros((m, n)), 1.0, 0.0).cpu().numpy()
    assert np.array_equal(got, float((v * w).sum()) * (u @ z.T))


def test_beta_zero_ignores_nan_c_and_alpha_zero_ignores_nan_ab():
    m, n, k = 65, 66, 67
    A, B, _ = host_mats(34, m, n, k)
    got = run(A, B, np.full((m, n), np.nan), 1.0, 0.0).cpu().numpy()
    assert np.isfinite(got).all()
    C = synth.matrix(34, 2, m, n)
    got = run(np.full((m, k), np.nan), np.full((k, n), np.nan), C, 0.0, 0.5).cpu().numpy()
    assert np.array_equal(got, 0.5 * C)
    got = run(None, None, C, 1.0, 2.0).cpu().numpy()  # k == 0
    assert np.array_equal(got, 2.0 * C)


def test_empty_is_noop():
    C = torch.full((0, 5), 1.0, dtype=torch.float64, device="cuda")
    mg.gemm(torch.empty(0, 3, dtype=torch.float64, device="cuda"),
            torch.empty(3, 5, dtype=torch.float64, device="cuda"), C)
    C = torch.full((4, 0), 1.0, dtype=torch.float64, device="cuda")
    mg.gemm(torch.empty(4, 3, dtype=torch.float64, device="cuda"),
            torch.empty(3, 0, dtype=torch.float64, device="cuda"), C)


def test_padded_ld_canaries_survive():
    m, n, k = 131, 77, 45
    A, B, C = host_mats(35, m, n, k)
    ldc = 96
    dC = to_dev(C, torch.float64, ldc, fill=12345.0)
    dA = to_dev(A, torch.float64, 64, fill=np.nan)
    dB = to_dev(B, torch.float64, 80, fill=np.nan)
    mg.gemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    parent = dC.as_strided((m, ldc), (ldc, 1)).cpu().numpy()
    assert (parent[:, n:] == 12345.0).all()
    check_f64(dC.cpu().numpy(), A, B, C, 1.0, 1.0, "padded ld")


def test_unaligned_operands_use_scalar_path():
    m, n, k = 67, 45, 33
    A, B, C = host_mats(36, m, n, k)
    # odd pitches and an 8-byte (not 16-byte) aligned base
    bigA = to_dev(np.zeros((m, k + 2)), torch.float64)
    dA = bigA[:, 1:k + 1]
    dA.copy_(torch.from_numpy(A))
    dB = to_dev(B, torch.float64, n + 1)
    dC = to_dev(C, torch.float64, n + 3)
    mg.gemm(dA, dB, dC, 1.0, 0.5)
    torch.cuda.synchronize()
    check_f64(dC.cpu().numpy(), A, B, C, 1.0, 0.5, "unaligned")


def test_paper_fill_range():
    """The paper's own fill: square, values in [0, 10]."""
    n = 384
    A = synth.matrix(37, 0, n, n, kind="paper")
    B = synth.matrix(37, 1, n, n, kind="paper")
    C = np.zeros((n, n))
    got = run(A, B, C, 1.0, 0.0).cpu().numpy()
    check_f64(got, A, B, C, 1.0, 0.0, "paper fill")


def test_deterministic_repeats():
    n = 640
    A, B, C = host_mats(38, n, n, n)
    dA, dB = to_dev(A), to_dev(B)
    outs = []
    for _ in range(3):
        dC = to_dev(C)
        mg.gemm(dA, dB, dC, 1.0, 1.0)
        outs.append(dC)
    torch.cuda.synchronize()
    assert all(torch.equal(outs[0], o) for o in outs[1:])


@pytest.mark.parametrize("cfg", [0, 2, 4, 5, 7, 9, 10, 12, 13])
@pytest.mark.parametrize("shape", [(33, 17, 65), (129, 130, 131), (256, 256, 256), (300, 200, 517)])
def test_native_f32_parity(cfg, shape):
    m, n, k = shape
    A, B, C = host_mats(39 + m, m, n, k)
    A32, B32, C32 = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
    got = run(A32, B32, C32, 1.0, 1.0, cfg=cfg, dtype=torch.float32).double().cpu().numpy()
    ref = oracle.dgemm(1.0, A32, B32, 1.0, C32)
    err = oracle.rel_fro_err(got, ref)
    bound = elementwise_bound(1.0, A32, B32, 1.0, C32, k, u=U32)
    log(f"f32 cfg{cfg} {shape}: rel_fro_err={err:.3e}")
    assert err <= 1e-5
    assert (np.abs(got - ref) <= bound).all()


@pytest.mark.parametrize("mnk", [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096),
                                 (8192, 8192, 8192), (8192, 1024, 4096), (1024, 8192, 8192)])
def test_config2_sizes_sampled(mnk):
    """Workload 2 at full size with the default work division (the bench's):
    sampled output rows/columns against the oracle, which computes each of
    them from one row of A and one column of B."""
    m, n, k = mnk
    log(f"config2 sampled {mnk}")
    seed = synth.config_seed(2)
    dA = synth.matrix(seed, synth.STREAM_A, m, k, device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, k, n, device="cuda")
    dC = synth.matrix(seed, synth.STREAM_C, m, n, device="cuda")
    C0 = dC.clone()
    mg.gemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    # log-uniform indices crowd the first tiles; uniform ones reach the last
    rows = np.unique(np.concatenate([[0, m - 1], synth.log_uniform_int(seed, 9, 40, 1, m - 1),
                                     (synth.uniform_unit(seed, 11, 40) * m).astype(np.int64)]))
    cols = np.unique(np.concatenate([[0, n - 1], synth.log_uniform_int(seed, 10, 40, 1, n - 1),
                                     (synth.uniform_unit(seed, 12, 40) * n).astype(np.int64)]))
    rt = torch.from_numpy(rows).cuda()
    ct = torch.from_numpy(cols).cuda()
    As = dA[rt].cpu().numpy()
    Bs = dB[:, ct].cpu().numpy()
    Cs = C0[rt][:, ct].cpu().numpy()
    got = dC[rt][:, ct].cpu().numpy()
    check_f64(got, As, Bs, Cs, 1.0, 1.0, f"config2 {mnk} sampled")
    assert torch.isfinite(dC).all()


@pytest.mark.parametrize("mnk", [(4096, 4096, 4096), (8192, 1024, 4096), (8192, 8192, 8192)])
def test_config2_full_output(mnk):
    """Workload 2 at full size with the bench's work division: every output
    element against the oracle (relative Frobenius error and the per-element
    rounding bound), including the headline n = 8192."""
    m, n, k = mnk
    log(f"config2 full {mnk}")
    seed = synth.config_seed(2)
    dA = synth.matrix(seed, synth.STREAM_A, m, k, device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, k, n, device="cuda")
    dC = synth.matrix(seed, synth.STREAM_C, m, n, device="cuda")
    C0 = dC.cpu().numpy()
    mg.gemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    A = dA.cpu().numpy()
    B = dB.cpu().numpy()
    del dA, dB
    check_f64(dC.cpu().numpy(), A, B, C0, 1.0, 1.0, f"config2 {mnk} full")


def test_metamorphic_transpose_bit_exact():
    """(A B)^T = B^T A^T: every output sums the same products in the same k
    order whichever operand feeds which side of the matrix core, so the two
    results agree bit for bit."""
    m, n, k = 300, 200, 517
    A, B, _ = host_mats(41, m, n, k)
    C1 = run(A, B, np.zeros((m, n)), 1.0, 0.0).cpu().numpy()
    C2 = run(np.ascontiguousarray(B.T), np.ascontiguousarray(A.T), np.zeros((n, m)), 1.0,
             0.0).cpu().numpy()
    assert np.array_equal(C1, C2.T)


def test_metamorphic_row_permutation_and_power_of_two_scaling():
    """Permuting the rows of A permutes the rows of C, and scaling A by 2^t
    scales C by 2^t, both bit for bit (each output's arithmetic depends only
    on its own row of A and column of B)."""
    m, n, k = 257, 190, 333
    A, B, _ = host_mats(42, m, n, k)
    perm = np.argsort(synth.uniform_unit(42, 9, m))
    base = run(A, B, np.zeros((m, n)), 1.0, 0.0).cpu().numpy()
    permuted = run(np.ascontiguousarray(A[perm]), B, np.zeros((m, n)), 1.0, 0.0).cpu().numpy()
    assert np.array_equal(permuted, base[perm])
    scaled = run(A * 2.0 ** 37, B, np.zeros((m, n)), 1.0, 0.0).cpu().numpy()
    assert np.array_equal(scaled, base * 2.0 ** 37)


def padded(cols):
    """A row pitch that keeps 16-byte rows for FP64 and FP32 and leaves padding."""
    return (cols + 7) // 8 * 8 + 8


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("cfg", DMA_CFGS)
@pytest.mark.parametrize("shape", [(33, 17, 65), (70, 45, 15), (129, 130, 131), (300, 200, 517),
                                   (256, 256, 256), (257, 129, 33)])
def test_native_dma_aligned_ragged(dt, cfg, shape):
    """Direct-to-LDS work divisions on 16-byte aligned operands with ragged m,
    n and k: the padding of A and B holds NaN (read by edge chunks, never
    allowed into a sum) and C's padding a canary that must survive."""
    m, n, k = shape
    A, B, C = host_mats(43 + m + n, m, n, k)
    dtype = torch.float64 if dt == "f64" else torch.float32
    if dt == "f32":
        A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
    dA = to_dev(A, dtype, padded(k))
    dB = to_dev(B, dtype, padded(n))
    dC = to_dev(C, dtype, padded(n), fill=12345.0)
    mg.gemm(dA, dB, dC, 1.5, 0.5, cfg=cfg)
    torch.cuda.synchronize()
    parent = dC.as_strided((m, padded(n)), (padded(n), 1)).cpu().numpy()
    assert (parent[:, n:] == 12345.0).all()
    got = dC.double().cpu().numpy()
    if dt == "f64":
        check_f64(got, A, B, C, 1.5, 0.5, f"dma cfg{cfg} {shape}")
    else:
        ref = oracle.dgemm(1.5, A, B, 0.5, C)
        assert oracle.rel_fro_err(got, ref) <= 1e-5
        assert (np.abs(got - ref) <= elementwise_bound(1.5, A, B, 0.5, C, k, u=U32)).all()


@pytest.mark.parametrize("cfg", [c for c in DMA_CFGS if c not in KGROUP_CFGS])
def test_native_dma_matches_register_staged_bitwise(cfg):
    """Both staging schemes run the same k order and epilogue: identical bits."""
    m, n, k = 300, 260, 333
    A, B, C = host_mats(44, m, n, k)
    outs = []
    for c in (cfg, 0):
        dC = to_dev(C, torch.float64, padded(n))
        mg.gemm(to_dev(A, torch.float64, padded(k)), to_dev(B, torch.float64, padded(n)), dC,
                1.0, 1.0, cfg=c)
        torch.cuda.synchronize()
        outs.append(dC.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("cfg", KGROUP_CFGS)
def test_native_kgroups_deterministic(cfg, dt):
    """Two k groups sum halves of each k-step and meet in a fixed order: the
    same bits on every run, and within the oracle's bound (FP64: checked
    against the exact product)."""
    m, n, k = 300, 260, 1000
    A, B, C = host_mats(45, m, n, k)
    dtype = torch.float64 if dt == "f64" else torch.float32
    if dt == "f32":
        A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
    outs = []
    for _ in range(3):
        dC = to_dev(C, dtype, padded(n))
        mg.gemm(to_dev(A, dtype, padded(k)), to_dev(B, dtype, padded(n)), dC, 1.0, 1.0, cfg=cfg)
        torch.cuda.synchronize()
        outs.append(dC.double().cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    if dt == "f64":
        check_f64(outs[0], A, B, C, 1.0, 1.0, f"kgroups cfg{cfg}")
    else:
        ref = oracle.dgemm(1.0, A, B, 1.0, C)
        assert (np.abs(outs[0] - ref) <= elementwise_bound(1.0, A, B, 1.0, C, k, u=U32)).all()
