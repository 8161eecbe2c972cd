"""Pins of the split-precision oracle (no GPU).

The split method (error-free integer slicing with power-of-two row/column
scales, exact slice products, FP64 recombination) is pinned by identities
that hold exactly, by brute-force integer arithmetic, and by its truncation
error bound relative to the exact product from the compensated FP64 oracle.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle import split


@pytest.mark.parametrize("kind", ["i8", "bf16"])
def test_scales_bound_rows_and_columns(kind):
    A = synth.matrix(20, synth.STREAM_A, 33, 57, kind="spread")
    E = split.split_scales(A, axis=1)
    mx = np.abs(A).max(axis=1)
    assert (mx < np.ldexp(1.0, E)).all() and (mx >= np.ldexp(0.5, E)).all()
    F = split.split_scales(A, axis=0)
    mx = np.abs(A).max(axis=0)
    assert (mx < np.ldexp(1.0, F)).all() and (mx >= np.ldexp(0.5, F)).all()
    Z = np.zeros((3, 4))
    assert (split.split_scales(Z, 1) == 0).all()


@pytest.mark.parametrize("kind", ["i8", "bf16"])
@pytest.mark.parametrize("s", [1, 3, 7, 9])
def test_slices_exact_decomposition(kind, s):
    """x == 2^E (sum_t x_t 2^-bt + r_s 2^-bs) exactly, |x_t| < 2^b, |r_s| < 1."""
    bits = split.SPLIT_BITS[kind]
    A = synth.matrix(21, synth.STREAM_A, 17, 40, kind="spread")
    E = split.split_scales(A, 1)
    S, r = split.split_slices(A, E, 1, s, bits)
    assert np.abs(S).max() <= 2 ** bits - 1
    assert np.abs(r).max() < 1.0
    # exact identity, evaluated with Python integers/fractions on a few entries
    from fractions import Fraction
    for i, p in [(0, 0), (5, 17), (16, 39), (3, 8)]:
        v = sum(Fraction(int(S[t, i, p]), 2 ** (bits * (t + 1))) for t in range(s))
        v += Fraction(float(r[i, p])) / 2 ** (bits * s)
        v *= Fraction(2) ** int(E[i])
        assert v == Fraction(float(A[i, p]))
    # reconstruction error below one unit of the last slice
    R = split.split_reconstruct(S, E, 1, bits)
    assert (np.abs(A - R) < np.ldexp(1.0, E[:, None] - bits * s)).all()


def test_slices_reconstruct_exactly_when_bits_suffice():
    """Entries within a factor 2 of the row max need 53 bits: 8 slices of 7."""
    A = synth.matrix(22, synth.STREAM_A, 9, 31)
    A = np.ldexp(np.sign(A) * (0.5 + 0.5 * np.abs(A)), 0)  # |a| in [0.5, 1)
    E = split.split_scales(A, 1)
    S, r = split.split_slices(A, E, 1, 8, 7)
    assert np.array_equal(split.split_reconstruct(S, E, 1, 7), A)
    assert (r == 0).all()


def test_products_brute_force_integers():
    """P_d against pure-Python integer sums for a tiny case."""
    s, bits = 4, 7
    A = synth.matrix(23, synth.STREAM_A, 3, 5, kind="spread")
    B = synth.matrix(23, synth.STREAM_B, 5, 4, kind="spread")
    As, _ = split.split_slices(A, split.split_scales(A, 1), 1, s, bits)
    Bs, _ = split.split_slices(B, split.split_scales(B, 0), 0, s, bits)
    P = split.split_products(As, Bs, bits)
    assert sorted(P) == list(range(2, s + 2))
    for d in range(2, s + 2):
        for i in range(3):
            for j in range(4):
                tot = 0
                for p in range(1, s + 1):
                    q = d - p
                    if 1 <= q <= s:
                        tot += sum(int(As[p - 1, i, t]) * int(Bs[q - 1, t, j]) for t in range(5))
                assert P[d][i, j] == tot


@pytest.mark.parametrize("kind", ["i8", "bf16"])
@pytest.mark.parametrize("s", [3, 5, 7])
def test_split_gemm_within_truncation_bound(kind, s):
    """|C_split - C_exact| <= |alpha| k 2^(E_i+F_j) (s+3) 2^(-bs) + rounding,
    per element, with the exact product from the compensated oracle."""
    bits = split.SPLIT_BITS[kind]
    m, n, k = 24, 20, 96
    A = synth.matrix(24, synth.STREAM_A, m, k, kind="spread")
    B = synth.matrix(24, synth.STREAM_B, k, n, kind="spread")
    C = synth.matrix(24, synth.STREAM_C, m, n)
    alpha, beta = 1.5, 0.5
    got = split.split_gemm(alpha, A, B, beta, C, s, kind)
    ref = oracle.dgemm(alpha, A, B, beta, C)
    E = split.split_scales(A, 1)
    F = split.split_scales(B, 0)
    scale = np.ldexp(1.0, E[:, None] + F[None, :])
    bound = abs(alpha) * k * scale * (s + 3) * 2.0 ** (-bits * s)
    bound += 8 * np.spacing(np.abs(ref)) + 4 * np.spacing(np.abs(alpha) * k * scale)
    assert (np.abs(got - ref) <= bound).all()


def test_split_gemm_error_falls_with_slices():
    m, n, k = 32, 32, 256
    A = synth.matrix(25, synth.STREAM_A, m, k, kind="spread")
    B = synth.matrix(25, synth.STREAM_B, k, n, kind="spread")
    ref = oracle.dgemm(1.0, A, B, 0.0, None)
    errs = [oracle.rel_fro_err(split.split_gemm(1.0, A, B, 0.0, None, s, "i8"), ref)
            for s in (3, 5, 7, 9)]
    assert errs[0] > errs[1] > errs[2] >= errs[3]
    assert errs[2] <= 1e-12
    assert errs[3] <= 1e-15


def test_split_gemm_small_integers_exact():
    """Integers in [-8, 8] fit in the first 7-bit slice of their row (column)
    scale, so every slice product and the recombination are exact."""
    A = synth.small_int_matrix(26, 0, 12, 30)
    B = synth.small_int_matrix(26, 1, 30, 9)
    C = synth.small_int_matrix(26, 2, 12, 9)
    got = split.split_gemm(1.5, A, B, 0.5, C, 3, "i8")
    assert np.array_equal(got, 1.5 * (A @ B) + 0.5 * C)
