"""Parity of the split-precision HIP path with the oracle (needs a GPU).

The scale and slice stages are exact integer work: the workspace the GPU
writes must equal the oracle's exponents and slices bit for bit, padding
included.  The slice products are exact integers too, and the recombination
and epilogue are specified operation by operation, so the GPU result must
equal the oracle's split result bit for bit (while k fits one exact INT32
segment); it must also be within 1e-12 relative Frobenius error of the exact
product from the compensated FP64 oracle.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import split as osplit
from helpers import SPLIT_CFGS, host_mats, log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")

ALGOS = {"i8": 1, "bf16": 2}


def spread(seed, m, n, k):
    A = synth.matrix(seed, synth.STREAM_A, m, k, kind="spread")
    B = synth.matrix(seed, synth.STREAM_B, k, n, kind="spread")
    C = synth.matrix(seed, synth.STREAM_C, m, n)
    return A, B, C


def decode_workspace(ws, L, s, m, n, k):
    raw = ws.cpu().numpy()
    E = raw[L["e_off"]: L["e_off"] + 4 * L["mp"]].view(np.int32)
    F = raw[L["f_off"]: L["f_off"] + 4 * L["np"]].view(np.int32)
    eb = L["elem_bytes"]
    a = raw[L["a_off"]: L["a_off"] + s * L["mp"] * L["kp"] * eb]
    b = raw[L["b_off"]: L["b_off"] + s * L["np"] * L["kp"] * eb]
    if eb == 1:
        As = a.view(np.int8).astype(np.int32)
        Bs = b.view(np.int8).astype(np.int32)
    else:  # bf16 bits -> float32 -> int
        As = (a.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.int32)
        Bs = (b.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.int32)
    As = As.reshape(s, L["mp"], L["kp"])
    Bs = Bs.reshape(s, L["np"], L["kp"])
    return E, F, As, Bs


@pytest.mark.parametrize("kind", ["i8", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (37, 45, 200), (130, 129, 257)])
@pytest.mark.parametrize("s", [1, 4, 7])
def test_slices_bit_exact(kind, shape, s):
    m, n, k = shape
    algo = ALGOS[kind]
    bits = osplit.SPLIT_BITS[kind]
    A, B, _ = spread(40 + m, m, n, k)
    L = mg.split_layout(algo, s, m, n, k)
    ws = torch.full((L["total_bytes"],), 0x5A, dtype=torch.uint8, device="cuda")
    mg.split_prepare(algo, s, to_dev(A), to_dev(B), ws)
    torch.cuda.synchronize()
    E, F, As, Bs = decode_workspace(ws, L, s, m, n, k)
    Eo = osplit.split_scales(A, 1)
    Fo = osplit.split_scales(B, 0)
    assert np.array_equal(E[:m], Eo) and (E[m:] == 0).all()
    assert np.array_equal(F[:n], Fo) and (F[n:] == 0).all()
    Ao, _ = osplit.split_slices(A, Eo, 1, s, bits)
    Bo, _ = osplit.split_slices(B, Fo, 0, s, bits)
    assert np.array_equal(As[:, :m, :k], Ao)
    assert np.array_equal(Bs[:, :n, :k], Bo.transpose(0, 2, 1))
    assert (As[:, m:, :] == 0).all() and (As[:, :, k:] == 0).all()
    assert (Bs[:, n:, :] == 0).all() and (Bs[:, :, k:] == 0).all()


@pytest.mark.parametrize("kind", ["i8", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 33, 64), (130, 129, 257), (256, 384, 700)])
def test_split_gemm_bit_exact_vs_oracle_split(kind, shape):
    m, n, k = shape
    algo = ALGOS[kind]
    s = mg.split_default_slices(algo)
    A, B, C = spread(50 + k, m, n, k)
    dC = to_dev(C)
    mg.gemm_split(to_dev(A), to_dev(B), dC, 1.5, 0.5, algo=algo, slices=s)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    want = osplit.split_gemm(1.5, A, B, 0.5, C, s, kind)
    ref = oracle.dgemm(1.5, A, B, 0.5, C)
    err = oracle.rel_fro_err(got, ref)
    log(f"split {kind} s={s} {shape}: rel_fro_err={err:.3e}")
    assert np.array_equal(got, want)
    assert err <= 1e-12


@pytest.mark.parametrize("kind", ["i8", "bf16"])
@pytest.mark.parametrize("s", [3, 5, 8])
def test_split_other_slice_counts(kind, s):
    m, n, k = 96, 160, 320
    algo = ALGOS[kind]
    A, B, C = spread(60 + s, m, n, k)
    dC = to_dev(C)
    mg.gemm_split(to_dev(A), to_dev(B), dC, 1.0, 1.0, algo=algo, slices=s)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), osplit.split_gemm(1.0, A, B, 1.0, C, s, kind))


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_split_long_k_segments(kind):
    """k beyond one exact INT32 segment: the kernel flushes each diagonal to
    FP64 per segment, so only the error bar applies (not bit equality)."""
    algo = ALGOS[kind]
    s = mg.split_default_slices(algo)
    m, n = 40, 48
    k = 20000 if kind == "i8" else 6000
    A, B, C = spread(70, m, n, k)
    dC = to_dev(C)
    mg.gemm_split(to_dev(A), to_dev(B), dC, 1.0, 0.0, algo=algo, slices=s)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    ref = oracle.dgemm(1.0, A, B, 0.0, None)
    assert oracle.rel_fro_err(got, ref) <= 1e-12
    want = osplit.split_gemm(1.0, A, B, 0.0, None, s, kind)
    assert oracle.rel_fro_err(got, want) <= 1e-14


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_split_small_integers_exact(kind):
    m, n, k = 70, 50, 90
    A = synth.small_int_matrix(71, 0, m, k)
    B = synth.small_int_matrix(71, 1, k, n)
    C = synth.small_int_matrix(71, 2, m, n)
    dC = to_dev(C)
    mg.gemm_split(to_dev(A), to_dev(B), dC, 1.5, 0.5, algo=ALGOS[kind], slices=2)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), 1.5 * (A @ B) + 0.5 * C)


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_split_special_cases(kind):
    algo = ALGOS[kind]
    m, n, k = 33, 35, 37
    A, B, C = spread(72, m, n, k)
    dC = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    mg.gemm_split(to_dev(A), to_dev(B), dC, 1.0, 0.0, algo=algo)
    torch.cuda.synchronize()
    assert torch.isfinite(dC).all()
    dC = to_dev(C)
    mg.gemm_split(to_dev(np.full((m, k), np.nan)), to_dev(np.full((k, n), np.nan)), dC, 0.0, 0.5,
                  algo=algo)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), 0.5 * C)
    zA = np.zeros((m, k))
    zA[5] = A[5]
    dC = to_dev(C)
    mg.gemm_split(to_dev(zA), to_dev(B), dC, 1.0, 1.0, algo=algo)
    torch.cuda.synchronize()
    s = mg.split_default_slices(algo)
    assert np.array_equal(dC.cpu().numpy(), osplit.split_gemm(1.0, zA, B, 1.0, C, s, kind))


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_pooled_workspace_matches_explicit(kind):
    algo = ALGOS[kind]
    m, n, k = 200, 190, 300
    A, B, C = spread(73, m, n, k)
    dA, dB = to_dev(A), to_dev(B)
    c1 = to_dev(C)
    c2 = to_dev(C)
    mg.gemm(dA, dB, c1, 1.0, 1.0, algo=algo)
    mg.gemm_split(dA, dB, c2, 1.0, 1.0, algo=algo)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2)


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_config3_n4096_sampled(kind):
    """Workload 3 at full size: n=4096, entries u*2^e with e in [-20, 20];
    sampled rows/columns against the exact product at the 1e-12 bar, and
    against the oracle's split result."""
    n = 4096
    algo = ALGOS[kind]
    s = mg.split_default_slices(algo)
    seed = synth.config_seed(3)
    log(f"config3 {kind} s={s}")
    dA = synth.matrix(seed, synth.STREAM_A, n, n, kind="spread", device="cuda")
    dB = synth.matrix(seed, synth.STREAM_B, n, n, kind="spread", device="cuda")
    dC = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    mg.gemm_split(dA, dB, dC, 1.0, 0.0, algo=algo, slices=s)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, n - 1], synth.log_uniform_int(seed, 9, 24, 1, n - 1)]))
    cols = np.unique(np.concatenate([[0, n - 1], synth.log_uniform_int(seed, 10, 24, 1, n - 1)]))
    rt, ct = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    A = dA.cpu().numpy()
    B = dB.cpu().numpy()
    got = dC[rt][:, ct].cpu().numpy()
    ref = oracle.dgemm(1.0, A[rows], B[:, cols], 0.0, None)
    err = oracle.rel_fro_err(got, ref)
    log(f"config3 {kind}: sampled rel_fro_err={err:.3e}")
    assert err <= 1e-12
    # the scales depend on whole rows/columns, the slices on single entries
    Eo = osplit.split_scales(A[rows], 1)
    Fo = osplit.split_scales(B[:, cols], 0)
    bits = osplit.SPLIT_BITS[kind]
    Ao, _ = osplit.split_slices(A[rows], Eo, 1, s, bits)
    Bo, _ = osplit.split_slices(B[:, cols], Fo, 0, s, bits)
    P = osplit.split_products(Ao, Bo, bits)
    acc = np.zeros((len(rows), len(cols)))
    for d in range(2, s + 2):
        acc = acc + np.ldexp(P[d], -bits * d)
    want = np.ldexp(acc, (Eo[:, None] + Fo[None, :]).astype(np.int32))
    assert np.array_equal(got, want)


def test_int8_default_large_ragged_matches_other_division_and_oracle():
    """INT8 single calls take the all-pairs 64x64 tile at every size: on a
    large ragged shape its result equals the 256x256 ring's (division 4) bit
    for bit, and sampled rows/columns equal the oracle's split result and
    lie within 1e-12 of the exact product."""
    m, n, k = 3000, 2500, 1100
    algo = ALGOS["i8"]
    s = mg.split_default_slices(algo)
    A, B, C = spread(61, m, n, k)
    dA, dB = to_dev(A), to_dev(B)
    c_pick, c_ring = to_dev(C), to_dev(C)
    mg.gemm(dA, dB, c_pick, 1.5, 0.5, algo=algo)
    mg.gemm_split(dA, dB, c_ring, 1.5, 0.5, algo=algo, slices=s, cfg=4)
    torch.cuda.synchronize()
    assert torch.equal(c_pick, c_ring)
    rows = np.unique(np.concatenate([[0, m - 1], synth.log_uniform_int(61, 9, 20, 1, m - 1)]))
    cols = np.unique(np.concatenate([[0, n - 1], synth.log_uniform_int(61, 10, 20, 1, n - 1)]))
    got = c_pick.cpu().numpy()[np.ix_(rows, cols)]
    Cs = C[np.ix_(rows, cols)]
    # row scales depend on whole rows of A, column scales on whole columns of B
    want = osplit.split_gemm(1.5, A[rows], B[:, cols], 0.5, Cs, s, "i8")
    assert np.array_equal(got, want)
    err = oracle.rel_fro_err(got, oracle.dgemm(1.5, A[rows], B[:, cols], 0.5, Cs))
    log(f"split i8 {(m, n, k)} default pick: sampled rel_fro_err={err:.3e}")
    assert err <= 1e-12


def test_workspace_below_operands_is_not_an_overlap():
    """Regression: a workspace at lower addresses than the operands (allocated
    first) was once reported as overlapping them."""
    m, n, k = 64, 80, 96
    algo = ALGOS["i8"]
    s = mg.split_default_slices(algo)
    ws = mg.split_workspace(algo, s, m, n, k)
    A, B, C = spread(74, m, n, k)
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
    mg.gemm_split(dA, dB, dC, 1.0, 1.0, algo=algo, slices=s, workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), osplit.split_gemm(1.0, A, B, 1.0, C, s, "i8"))


@pytest.mark.parametrize("kind", ["i8", "bf16"])
@pytest.mark.parametrize("cfg", list(range(SPLIT_CFGS)))
def test_split_work_divisions_bit_exact(kind, cfg):
    """Every work division of the product kernel gives the oracle's bits."""
    algo = ALGOS[kind]
    s = mg.split_default_slices(algo)
    m, n, k = 300, 520, 384
    A, B, C = spread(75 + cfg, m, n, k)
    dC = to_dev(C)
    mg.gemm_split(to_dev(A), to_dev(B), dC, 1.5, -0.5, algo=algo, slices=s, cfg=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), osplit.split_gemm(1.5, A, B, -0.5, C, s, kind))


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_split_row_permutation_and_power_of_two_scaling(kind):
    """A row's exponent, slices and products depend only on that row, so
    permuting the rows of A permutes the rows of C and scaling a row of A by
    2^t scales the same row of C (beta = 0), bit for bit."""
    m, n, k = 200, 150, 300
    algo = ALGOS[kind]
    s = mg.split_default_slices(algo)
    A, B, _ = spread(61, m, n, k)

    def go(Ax):
        dC = torch.zeros(m, n, dtype=torch.float64, device="cuda")
        mg.gemm_split(to_dev(Ax), to_dev(B), dC, 1.0, 0.0, algo=algo, slices=s)
        torch.cuda.synchronize()
        return dC.cpu().numpy()

    base = go(A)
    perm = np.argsort(synth.uniform_unit(61, 9, m))
    assert np.array_equal(go(np.ascontiguousarray(A[perm])), base[perm])
    t = np.arange(m) % 7 - 3  # per-row power-of-two scale factors
    assert np.array_equal(go(A * np.ldexp(1.0, t)[:, None]), base * np.ldexp(1.0, t)[:, None])


@pytest.mark.parametrize("kind", ["i8", "bf16"])
@pytest.mark.parametrize("shape,s", [((1792, 1700, 256), None), ((700, 650, 300), None),
                                     ((100, 90, 20000), None), ((64, 80, 96), 1),
                                     ((64, 80, 96), 2), ((200, 150, 130), 16)])
def test_pair_parallel_matches_fused(kind, shape, s):
    """The pair-parallel division (15: groups of slice pairs x 128x128 tiles,
    then the fold) gives the fused register-staged division's bits, across
    group counts (2 to 28 groups), several k segments (k = 20000) and slice
    counts 1, 2 and 16."""
    m, n, k = shape
    algo = ALGOS[kind]
    default = s is None
    s = s or mg.split_default_slices(algo)
    A, B, C = spread(80 + m % 97, m, n, k)
    dA, dB = to_dev(A), to_dev(B)
    out = []
    for cfg in (0, 15):
        dC = to_dev(C)
        mg.gemm_split(dA, dB, dC, 1.25, 0.75, algo=algo, slices=s, cfg=cfg)
        torch.cuda.synchronize()
        out.append(dC.cpu().numpy())
    log(f"pairs vs fused {kind} s={s} {shape}: equal={np.array_equal(out[0], out[1])}")
    assert np.array_equal(out[0], out[1])
    if default and m * n * k <= 100 * 90 * 20000:
        ref = oracle.dgemm(1.25, A, B, 0.75, C)
        assert oracle.rel_fro_err(out[1], ref) <= 1e-12
