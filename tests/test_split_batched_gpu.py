"""Batched split-precision GEMM (mg_gemm_batched with MG_SPLIT_I8 / BF16).

Every problem of a batch must come out bit for bit as mg_gemm with the same
algorithm gives it alone (the batched launches run the fused division's tile
code; slices and integer products are exact and the fold order is fixed),
and, while k fits one exact INT32 segment, bit for bit as the oracle's split
result; beyond one segment within 1e-14 of it and 1e-12 of the exact
product.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import split as osplit
from helpers import log, make_batch, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")

ALGOS = {"i8": mg.SPLIT_I8, "bf16": mg.SPLIT_BF16}
# k of one exact INT32 segment at the default slice counts (7 / 6): whole
# 128-byte stages with s * k_seg * (2^b - 1)^2 < 2^31 (BF16: whole 256-k chunks)
SEGMENT_K = {"i8": 148 * 128, "bf16": 84 * 64}


def spread(seed, m, n, k):
    A = synth.matrix(seed, synth.STREAM_A, m, k, kind="spread")
    B = synth.matrix(seed, synth.STREAM_B, k, n, kind="spread")
    C = synth.matrix(seed, synth.STREAM_C, m, n)
    return A, B, C


def mixed_cases(kind):
    """(m, n, k, alpha, beta, lda pad, ldc pad): ragged tiles, several tiles
    per problem, one past an INT32 segment, padded rows, degenerate ones."""
    long_k = 20000 if kind == "i8" else 6000
    return [
        (1, 1, 1, 1.0, 0.0, 0, 0),
        (17, 33, 64, 1.5, 0.5, 0, 0),
        (130, 129, 257, 1.0, 1.0, 3, 0),
        (256, 384, 700, -0.75, 0.25, 0, 5),
        (300, 20, 1000, 1.0, 0.0, 0, 0),
        (20, 300, 129, 2.0, -1.0, 0, 0),
        (40, 48, long_k, 1.0, 0.5, 0, 0),
        (64, 64, 0, 1.0, 0.5, 0, 0),      # k = 0: C <- beta*C
        (50, 60, 70, 0.0, 0.5, 0, 0),     # alpha = 0: C <- beta*C
        (0, 40, 30, 1.0, 1.0, 0, 0),      # empty
        (129, 1, 513, 1.0, 0.0, 0, 0),
        (1, 257, 100, 1.0, 1.0, 0, 0),
    ]


def run_cases(kind, cases, seed0):
    algo = ALGOS[kind]
    ops, probs, C_single, C_batch, keep = [], [], [], [], []
    for i, (m, n, k, alpha, beta, pa, pc) in enumerate(cases):
        A, B, C = spread(seed0 + i, m, n, k)
        dA = to_dev(A, ld=k + pa if pa else None)
        dB = to_dev(B)
        keep += [dA, dB]  # descriptors hold raw pointers: keep the operands alive
        c1 = to_dev(C, ld=n + pc if pc else None)
        c2 = to_dev(C, ld=n + pc if pc else None)
        ops.append((A, B, C, alpha, beta))
        C_single.append(c1)
        C_batch.append(c2)
        probs.append(mg.problem(dA, dB, c2, alpha, beta))
        if m and n:
            mg.gemm(dA, dB, c1, alpha, beta, algo=algo)
    mg.gemm_batched(probs, dtype=mg.F64, algo=algo)
    torch.cuda.synchronize()
    del keep
    return ops, C_single, C_batch


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_batched_split_matches_single_and_oracle(kind):
    algo = ALGOS[kind]
    s = mg.split_default_slices(algo)
    cases = mixed_cases(kind)
    ops, C_single, C_batch = run_cases(kind, cases, 900)
    for (m, n, k, alpha, beta, _, _), (A, B, C, _, _), c1, c2 in zip(cases, ops, C_single,
                                                                     C_batch):
        assert torch.equal(c1, c2), f"{kind} {(m, n, k)}: batched differs from single"
        if m == 0 or n == 0:
            continue
        got = c2.cpu().numpy()
        want = osplit.split_gemm(alpha, A, B, beta, C, s, kind)
        if k <= SEGMENT_K[kind]:
            assert np.array_equal(got, want), f"{kind} {(m, n, k)} vs oracle split"
        else:
            assert oracle.rel_fro_err(got, want) <= 1e-14
        ref = oracle.dgemm(alpha, A, B, beta, C)
        err = oracle.rel_fro_err(got, ref)
        assert err <= 1e-12, f"{kind} {(m, n, k)}: {err:.3e}"
    log(f"batched split {kind}: {len(cases)} problems bit-identical to single calls")


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_batched_split_config4_shapes(kind):
    """The 2000-problem batch workload (m, n, k log-uniform in [16, 512],
    beta = 1): every problem equal to its single call, 1 in 25 against the
    oracle's split result."""
    algo = ALGOS[kind]
    s = mg.split_default_slices(algo)
    shapes = [tuple(int(x) for x in sh) for sh in synth.batch_shapes(777, 2000)]
    views, flats, probs = make_batch(777, shapes)
    C0 = flats["C"].clone()
    mg.gemm_batched(probs, dtype=mg.F64, algo=algo)
    torch.cuda.synchronize()
    batched = flats["C"].clone()
    flats["C"].copy_(C0)
    for (A, B, C) in views:
        mg.gemm(A, B, C, 1.0, 1.0, algo=algo)
    torch.cuda.synchronize()
    assert torch.equal(batched, flats["C"]), "batched differs from single calls"
    flats["C"].copy_(C0)
    checked = 0
    for i in range(0, len(shapes), 25):
        A, B, C = views[i]
        want = osplit.split_gemm(1.0, A.cpu().numpy(), B.cpu().numpy(), 1.0, C.cpu().numpy(),
                                 s, kind)
        m, n, k = shapes[i]
        start = C.storage_offset() - flats["C"].storage_offset()  # this C in the saved copy
        got = batched[start: start + m * n].view(m, n).cpu().numpy()
        assert np.array_equal(got, want), f"problem {i} {shapes[i]}"
        checked += 1
    log(f"config4 split {kind}: 2000 problems equal to single calls, {checked} vs oracle")


def test_batched_split_repeat_reads_current_operands():
    """Nothing is cached between split batches: a second call with changed
    operands in the same buffers gives the new product, also after the
    workspace pool was trimmed."""
    shapes = [(70, 90, 110), (200, 130, 60)]
    views, flats, probs = make_batch(778, shapes, beta=0.0)
    mg.gemm_batched(probs, dtype=mg.F64, algo=mg.SPLIT_I8)
    torch.cuda.synchronize()
    flats["A"].mul_(2.0)
    mg.release_cached_memory()  # the workspace pool gives its blocks back; the next call
    mg.gemm_batched(probs, dtype=mg.F64, algo=mg.SPLIT_I8)  # allocates afresh
    torch.cuda.synchronize()
    for (A, B, C) in views:
        want = osplit.split_gemm(1.0, A.cpu().numpy(), B.cpu().numpy(), 0.0, None, 7, "i8")
        assert np.array_equal(C.cpu().numpy(), want)
