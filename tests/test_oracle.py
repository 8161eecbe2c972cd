"""Pins of the CPU oracle against facts fixed by mathematics (no GPU).

The oracle computes C <- alpha*A*B + beta*C (Section 4.2 of the Alpaka paper)
with compensated dot products.  None of these tests re-types its formula:
each compares it with an independent fact (exact rational arithmetic, closed
forms of structured products, exactness of small-integer arithmetic,
cancellation a plain sum gets wrong) chosen so that a dropped term, a wrong
sign, a transposed operand or an off-by-one in k fails at least one of them
(the mutation tests at the end check exactly that).
"""

import itertools
import math
import os
import shutil
import subprocess
import ctypes

import numpy as np
import pytest

import oracle
import synth


def ulp_diff(x, y):
    """|x - y| in units of the larger ulp (elementwise)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sp = np.maximum(np.spacing(np.abs(x)), np.spacing(np.abs(y)))
    return np.abs(x - y) / sp


# ----------------------------------------------------------- brute force n<=8
def test_brute_force_rational_all_shapes_to_8():
    """Every (m, n, k) in [1, 8]^3: oracle within 1 ulp of the exactly
    rounded rational result, and exactly equal in nearly all elements."""
    total = exact = 0
    worst = 0.0
    for m, n, k in itertools.product(range(1, 9), repeat=3):
        seed = synth.config_seed(0, 100 * m + 10 * n + k)
        A = synth.matrix(seed, synth.STREAM_A, m, k)
        B = synth.matrix(seed, synth.STREAM_B, k, n)
        C = synth.matrix(seed, synth.STREAM_C, m, n)
        R = oracle.dgemm(1.5, A, B, 0.5, C)
        X = oracle.exact_gemm(1.5, A, B, 0.5, C)
        d = ulp_diff(R, X)
        worst = max(worst, float(d.max()))
        total += d.size
        exact += int((d == 0).sum())
    assert worst <= 1.0, worst
    assert exact / total >= 0.999, (exact, total)


def test_exhaustive_ternary_2x2x2():
    """All 3^8 choices of A, B in {-1,0,1}^(2x2): integers, so exact."""
    C = np.array([[0.25, -3.0], [7.5, 1.0]])
    vals = (-1.0, 0.0, 1.0)
    for combo in itertools.product(vals, repeat=8):
        A = np.array(combo[:4]).reshape(2, 2)
        B = np.array(combo[4:]).reshape(2, 2)
        R = oracle.dgemm(2.0, A, B, -0.5, C)
        want = np.empty((2, 2))
        for i in range(2):
            for j in range(2):
                want[i, j] = 2.0 * (A[i, 0] * B[0, j] + A[i, 1] * B[1, j]) - 0.5 * C[i, j]
        assert np.array_equal(R, want), (A, B, R, want)


def test_exhaustive_ternary_1x1x1_with_beta_cases():
    for a, b, c in itertools.product((-1.0, 0.0, 1.0), repeat=3):
        for alpha, beta in ((1.0, 0.0), (1.5, 0.5), (-2.0, 1.0), (0.0, 3.0)):
            R = oracle.dgemm(alpha, np.array([[a]]), np.array([[b]]), beta, np.array([[c]]))
            assert R[0, 0] == alpha * a * b + beta * c


# ------------------------------------------------------------- closed forms
def test_identity():
    n = 37
    B = synth.matrix(7, synth.STREAM_B, n, 29)
    C0 = synth.matrix(7, synth.STREAM_C, n, 29)
    R = oracle.dgemm(1.0, np.eye(n), B, 0.0, None)
    assert np.array_equal(R, B)
    R = oracle.dgemm(1.5, np.eye(n), B, 0.5, C0)
    X = oracle.exact_gemm(1.5, np.eye(n)[:8, :8], B[:8], 0.5, C0[:8])
    assert ulp_diff(R[:8], X).max() == 0
    assert ulp_diff(R, 1.5 * B + 0.5 * C0).max() <= 1.0


def test_diagonal():
    n = 23
    d1 = synth.uniform_pm1(8, 0, n)
    d2 = synth.uniform_pm1(8, 1, n)
    C0 = synth.matrix(8, synth.STREAM_C, n, n)
    R = oracle.dgemm(-1.25, np.diag(d1), np.diag(d2), 0.75, C0)
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(R[off], (0.75 * C0)[off])
    X = oracle.exact_gemm(-1.25, np.diag(d1[:6]), np.diag(d2[:6]), 0.75, C0[:6, :6])
    assert ulp_diff(np.diag(R)[:6], np.diag(X)).max() == 0


def test_rank_one_small_integers():
    """A = u v^T, B = w z^T: A B = (v . w) u z^T, all exact integers."""
    m, k, n = 19, 41, 13
    u = synth.small_int_matrix(9, 0, m, 1)
    v = synth.small_int_matrix(9, 1, k, 1)
    w = synth.small_int_matrix(9, 2, k, 1)
    z = synth.small_int_matrix(9, 3, n, 1)
    A = u @ v.T
    B = w @ z.T
    vw = float((v[:, 0] * w[:, 0]).sum())
    R = oracle.dgemm(1.0, A, B, 0.0, None)
    assert np.array_equal(R, vw * (u @ z.T))


def test_small_integer_bit_exact():
    """Entries in [-8, 8], alpha=1.5, beta=0.5: every partial sum is exact, so
    the unique correct answer is the plain float product."""
    m, n, k = 65, 47, 130
    A = synth.small_int_matrix(10, 0, m, k)
    B = synth.small_int_matrix(10, 1, k, n)
    C = synth.small_int_matrix(10, 2, m, n)
    R = oracle.dgemm(1.5, A, B, 0.5, C)
    want = np.zeros((m, n))
    for p in range(k):  # exact in any order
        want += np.outer(A[:, p], B[p, :])
    assert np.array_equal(R, 1.5 * want + 0.5 * C)


# --------------------------------------------------------- compensation
def test_cancellation_needs_compensation():
    """2^60 + 1 - 2^60 = 1: a plain FP64 sum returns 0."""
    a = np.array([[2.0 ** 60, 1.0, -(2.0 ** 60)]])
    b = np.ones((3, 1))
    assert oracle.dgemm(1.0, a, b, 0.0, None)[0, 0] == 1.0
    # product errors too: (1+2^-30)^2 - 1 - 2^-29 = 2^-60 exactly
    x = 1.0 + 2.0 ** -30
    a = np.array([[x, -1.0, -(2.0 ** -29)]])
    b = np.array([[x], [1.0], [1.0]])
    assert oracle.dgemm(1.0, a, b, 0.0, None)[0, 0] == 2.0 ** -60


def test_ill_conditioned_random_dots():
    """Dot products built to cancel to a known small exact value."""
    rng_vals = synth.uniform_pm1(11, 0, 200)
    for t in range(20):
        big = rng_vals[10 * t: 10 * t + 5] * 2.0 ** 40
        small = rng_vals[10 * t + 5: 10 * t + 10]
        x = np.concatenate([big, small, -big])[None, :]
        y = np.ones((15, 1))
        exact = math.fsum(small.tolist())
        assert oracle.dgemm(1.0, x, y, 0.0, None)[0, 0] == exact


# ------------------------------------------------------ special cases (BLAS)
def test_beta_zero_does_not_read_c():
    A = synth.matrix(12, 0, 5, 6)
    B = synth.matrix(12, 1, 6, 7)
    C = np.full((5, 7), np.nan)
    R = oracle.dgemm(1.0, A, B, 0.0, C)
    assert np.isfinite(R).all()


def test_alpha_zero_and_k_zero():
    C = synth.matrix(13, 2, 4, 5)
    A = np.full((4, 3), np.nan)
    B = np.full((3, 5), np.nan)
    assert np.array_equal(oracle.dgemm(0.0, A, B, 0.5, C), 0.5 * C)
    assert np.array_equal(oracle.dgemm(1.0, None, None, 2.0, C, k=0), 2.0 * C)
    assert np.array_equal(oracle.dgemm(1.0, None, None, 0.0, np.full((4, 5), np.nan), k=0),
                          np.zeros((4, 5)))


def test_empty():
    assert oracle.dgemm(1.0, np.zeros((0, 3)), np.zeros((3, 4)), 0.0, None).shape == (0, 4)


def test_sampled_matches_full():
    A = synth.matrix(14, 0, 64, 50)
    B = synth.matrix(14, 1, 50, 70)
    C = synth.matrix(14, 2, 64, 70)
    R = oracle.dgemm(1.0, A, B, 1.0, C)
    rows = np.array([0, 5, 63])
    cols = np.array([69, 1, 2, 33])
    assert np.array_equal(oracle.dgemm_sampled(1.0, A, B, 1.0, C, rows, cols),
                          R[np.ix_(rows, cols)])


def test_paper_range_fill():
    """The paper's own fill (values in [0, 10]): all-positive, no cancellation."""
    A = synth.matrix(15, 0, 8, 8, kind="paper")
    B = synth.matrix(15, 1, 8, 8, kind="paper")
    assert A.min() >= 0.0 and A.max() < 10.0
    R = oracle.dgemm(1.0, A, B, 0.0, None)
    assert ulp_diff(R, oracle.exact_gemm(1.0, A, B, 0.0, None)).max() <= 1.0


def test_rel_fro_err():
    R = np.array([[3.0, 4.0]])
    assert oracle.rel_fro_err(R, R) == 0.0
    assert oracle.rel_fro_err(np.array([[3.0, 4.0 + 5.0]]), R) == 1.0
    assert oracle.rel_fro_err(np.array([[0.0, 2.0]]), np.zeros((1, 2))) == 2.0


# ------------------------------------------------------------ mutation tests
MUTATIONS = {
    "drop_compensation": ("c[j] += serr + perr;", "c[j] += 0.0 * (serr + perr);"),
    "beta_sign": ("two_prod(beta, *cij, &p2, &e2);", "two_prod(-beta, *cij, &p2, &e2);"),
    "k_off_by_one": ("for (int64_t p = 0; p < k; ++p) {", "for (int64_t p = 1; p < k; ++p) {"),
    "transposed_b": ("two_prod(a, brow[j], &prod, &perr);",
                     "two_prod(a, B[j * ldb + p], &prod, &perr);"),
}


def _pin_suite(lib):
    """Square cases only (the transposed mutation must stay in bounds)."""
    dp = ctypes.POINTER(ctypes.c_double)
    f = lib.oracle_dgemm
    f.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_double, dp, ctypes.c_int64, dp, ctypes.c_int64,
                                         ctypes.c_double, dp, ctypes.c_int64]

    def run(alpha, A, B, beta, C):
        out = np.array(C, dtype=np.float64, copy=True)
        A = np.ascontiguousarray(A)
        B = np.ascontiguousarray(B)
        n = A.shape[0]
        f(n, n, n, alpha, A.ctypes.data_as(dp), n, B.ctypes.data_as(dp), n, beta,
          out.ctypes.data_as(dp), n)
        return out

    ok = True
    for n in (3, 6):
        A = synth.matrix(16 + n, 0, n, n)
        B = synth.matrix(16 + n, 1, n, n)
        C = synth.matrix(16 + n, 2, n, n)
        ok &= ulp_diff(run(1.5, A, B, 0.5, C), oracle.exact_gemm(1.5, A, B, 0.5, C)).max() <= 1.0
    a = np.zeros((3, 3))
    a[0] = [2.0 ** 60, 1.0, -(2.0 ** 60)]
    ok &= run(1.0, a, np.ones((3, 3)), 0.0, np.zeros((3, 3)))[0, 0] == 1.0
    return bool(ok)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistakes(name, tmp_path):
    """Plant one plausible mistake in a copy of the oracle's C source (on the
    CPU) and check that the pins above fail for it."""
    from oracle import build as ob
    src = open(ob.SRC).read()
    old, new = MUTATIONS[name]
    assert old in src
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", *ob.CFLAGS, str(mutated), "-o", str(so), "-lm"], check=True)
    assert not _pin_suite(ctypes.CDLL(str(so))), name


def test_unmutated_oracle_passes_pin_suite():
    assert _pin_suite(ctypes.CDLL(oracle.LIB_PATH))
