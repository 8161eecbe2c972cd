"""Transposed operand layouts of the native kernels (mg_gemm_ex), needs a GPU.

C <- alpha*op(A)*op(B) + beta*C with A stored k x m (op(A) = A^T) and/or B
stored n x k (op(B) = B^T).  The oracle is the plain definition on the
logical matrices; the stored ones are their transposed copies.  Bars: FP64
relative Frobenius error <= 1e-13 and the per-element rounding bound; FP32
<= 1e-5 on FP32-rounded inputs; and, since the transposed layouts feed the
matrix cores the same products in the same k order, bit-identical results
to the plain layout with the same work division.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import DMA_CFGS, NATIVE_CFGS, U32, elementwise_bound, host_mats, log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")

LAYOUTS = [(1, 0), (0, 1), (1, 1)]
DTYPES = {"f64": torch.float64, "f32": torch.float32}


def stored(X, trans):
    return np.ascontiguousarray(X.T) if trans else X


def padded(cols, aligned):
    """Row pitch with padding: a multiple of 8 elements (16-byte rows for
    FP64 and FP32) when aligned, odd otherwise (element-wise loads)."""
    return (cols + 7) // 8 * 8 + 8 if aligned else (cols + 3) | 1


def run_ex(A, B, C, alpha, beta, ta, tb, cfg, dtype, aligned):
    sA, sB = stored(A, ta), stored(B, tb)
    dA = to_dev(sA, dtype, padded(sA.shape[1], aligned))
    dB = to_dev(sB, dtype, padded(sB.shape[1], aligned))
    dC = to_dev(C, dtype, padded(C.shape[1], aligned), fill=12345.0)
    mg.gemm_ex(dA, dB, dC, alpha, beta, transa=bool(ta), transb=bool(tb), cfg=cfg)
    torch.cuda.synchronize()
    return dC


def check(got, A, B, C, alpha, beta, dt, tag):
    ref = oracle.dgemm(alpha, A, B, beta, C)
    err = oracle.rel_fro_err(got, ref)
    u = 2.0 ** -53 if dt == "f64" else U32
    bound = elementwise_bound(alpha, A, B, beta, C, A.shape[1], u=u)
    log(f"{tag}: rel_fro_err={err:.3e}")
    assert err <= (1e-13 if dt == "f64" else 1e-5), (tag, err)
    assert (np.abs(got - ref) <= bound).all(), tag


def host_inputs(seed, m, n, k, dt):
    A, B, C = host_mats(seed, m, n, k)
    if dt == "f32":
        A, B, C = (x.astype(np.float32).astype(np.float64) for x in (A, B, C))
    return A, B, C


@pytest.mark.parametrize("aligned", [True, False])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("ta,tb", LAYOUTS)
@pytest.mark.parametrize("cfg", range(NATIVE_CFGS))
def test_transposed_every_cfg_matches_plain_bitwise_and_oracle(cfg, ta, tb, dt, aligned):
    """Every work division, both staging schemes (16-byte pitches take the
    direct-load rings for cfgs 14-24, odd pitches the register-staged
    tiles), ragged m, n and k; C's padding holds a canary."""
    m, n, k = 200, 136, 300
    log(f"trans cfg={cfg} ta={ta} tb={tb} {dt} aligned={aligned}")
    A, B, C = host_inputs(synth.config_seed(1, 60) + cfg, m, n, k, dt)
    dtype = DTYPES[dt]
    got = run_ex(A, B, C, 1.5, 0.5, ta, tb, cfg, dtype, aligned)
    plain = run_ex(A, B, C, 1.5, 0.5, 0, 0, cfg, dtype, aligned)
    assert torch.equal(got, plain)
    pitch = padded(n, aligned)
    parent = got.as_strided((m, pitch), (pitch, 1)).cpu().numpy()
    assert (parent[:, n:] == 12345.0).all()
    check(got.double().cpu().numpy(), A, B, C, 1.5, 0.5, dt, f"cfg{cfg} t{ta}{tb} {dt}")


SHAPES = [(1, 1, 1), (7, 5, 3), (8, 4, 6), (33, 17, 65), (70, 45, 15), (129, 130, 131),
          (64, 256, 31), (300, 200, 517), (257, 129, 33)]


@pytest.mark.parametrize("aligned", [True, False])
@pytest.mark.parametrize("ta,tb", LAYOUTS)
@pytest.mark.parametrize("cfg", sorted(set(DMA_CFGS) | {0, 2, 3, 4, 13}))
@pytest.mark.parametrize("shape", SHAPES)
def test_transposed_shapes_f64(shape, cfg, ta, tb, aligned):
    """Tiny, ragged and multi-tile shapes (tail k below one 16-byte chunk,
    m or n below one tile and below one chunk), the operands' padding NaN."""
    m, n, k = shape
    A, B, C = host_inputs(61 + m + 3 * n + 7 * k, m, n, k, "f64")
    got = run_ex(A, B, C, 1.5, 0.5, ta, tb, cfg, torch.float64, aligned)
    check(got.cpu().numpy(), A, B, C, 1.5, 0.5, "f64", f"cfg{cfg} t{ta}{tb} {shape}")


@pytest.mark.parametrize("ta,tb", LAYOUTS)
def test_transposed_special_cases(ta, tb):
    """beta == 0 never reads C (NaN stays out); alpha == 0 and k == 0 leave
    beta*C without reading A or B; empty outputs are no-ops."""
    m, n, k = 65, 66, 67
    A, B, _ = host_mats(62, m, n, k)
    got = run_ex(A, B, np.full((m, n), np.nan), 1.0, 0.0, ta, tb, None, torch.float64, True)
    assert torch.isfinite(got).all()
    C = synth.matrix(62, 2, m, n)
    nanA, nanB = np.full((m, k), np.nan), np.full((k, n), np.nan)
    got = run_ex(nanA, nanB, C, 0.0, 0.5, ta, tb, None, torch.float64, True).cpu().numpy()
    assert np.array_equal(got, 0.5 * C)
    dC = torch.from_numpy(C).cuda()
    mg.gemm_ex(torch.empty(0, m, dtype=torch.float64, device="cuda") if ta else
               torch.empty(m, 0, dtype=torch.float64, device="cuda"),
               torch.empty(n, 0, dtype=torch.float64, device="cuda") if tb else
               torch.empty(0, n, dtype=torch.float64, device="cuda"),
               dC, 1.0, 2.0, transa=bool(ta), transb=bool(tb))
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), 2.0 * C)


@pytest.mark.parametrize("ta,tb", LAYOUTS)
def test_transposed_small_integers_bit_exact(ta, tb):
    m, n, k = 150, 97, 301
    A = synth.small_int_matrix(63, 0, m, k)
    B = synth.small_int_matrix(63, 1, k, n)
    C = synth.small_int_matrix(63, 2, m, n)
    got = run_ex(A, B, C, 1.5, 0.5, ta, tb, None, torch.float64, True).cpu().numpy()
    assert np.array_equal(got, 1.5 * (A @ B) + 0.5 * C)


@pytest.mark.parametrize("ta,tb", LAYOUTS)
def test_transposed_full_size_sampled(ta, tb):
    """m = n = k = 8192 (the headline shape) with the default work division:
    bit-identical to the plain layout over the whole output, and sampled
    outputs against the oracle (one row of op(A), one column of op(B) each)."""
    n = 8192
    log(f"trans full size ta={ta} tb={tb}")
    seed = synth.config_seed(2)
    dA = synth.matrix(seed, synth.STREAM_A, n, n, device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, n, n, device="cuda")
    dC0 = synth.matrix(seed, synth.STREAM_C, n, n, device="cuda")
    plain = dC0.clone()
    mg.gemm(dA, dB, plain, 1.0, 1.0)
    sA = dA.t().contiguous() if ta else dA
    sB = dB.t().contiguous() if tb else dB
    got = dC0.clone()
    mg.gemm_ex(sA, sB, got, 1.0, 1.0, transa=bool(ta), transb=bool(tb))
    torch.cuda.synchronize()
    assert torch.equal(got, plain)
    rows = np.unique(np.concatenate([[0, n - 1], synth.log_uniform_int(seed, 9, 24, 1, n - 1)]))
    cols = np.unique(np.concatenate([[0, n - 1], synth.log_uniform_int(seed, 10, 24, 1, n - 1)]))
    rt, ct = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    As = (sA[:, rt].t() if ta else sA[rt]).cpu().numpy()
    Bs = (sB[ct].t() if tb else sB[:, ct]).cpu().numpy()
    Cs = dC0[rt][:, ct].cpu().numpy()
    check(got[rt][:, ct].cpu().numpy(), As, Bs, Cs, 1.0, 1.0, "f64", f"8192 t{ta}{tb} sampled")
