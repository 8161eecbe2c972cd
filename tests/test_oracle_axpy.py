"""Pins of the DAXPY oracle, y <- alpha*x + y (Section 4.1), no GPU.

Each element must be the exact value alpha*x[i] + y[i] rounded once to the
nearest double.  The pins compare with facts the oracle does not compute
itself: exact rational evaluation (Python fractions), hand-made cases whose
correct rounding is known in closed form (a product whose low part survives
only when it is not rounded first, ties to even), IEEE special values, the
BLAS quick return and the increments.  Planted mistakes in a copy of the C
source (unfused multiply-add, a dropped or sign-flipped term, a wrong
increment) must fail them.
"""

import ctypes
import subprocess

import numpy as np
import pytest

import oracle
import synth


def test_exact_rational_random_and_wide_exponents():
    n = 4000
    x = synth.exp_spread(71, 0, 1, n, -60, 60)
    y = synth.exp_spread(71, 2, 3, n, -60, 60)
    for alpha in (1.0, -0.75, 3.0e-5, 1.0 + 2.0 ** -40):
        assert np.array_equal(oracle.daxpy(alpha, x, y), oracle.exact_axpy(alpha, x, y)), alpha


def test_cancellation_exposes_a_rounded_product():
    """(1 + 2^-30)^2 - (1 + 2^-29) = 2^-60 exactly; rounding the product
    first loses it and gives 0."""
    a = 1.0 + 2.0 ** -30
    got = oracle.daxpy(a, np.array([a]), np.array([-(1.0 + 2.0 ** -29)]))
    assert got[0] == 2.0 ** -60


def test_ties_round_to_even():
    # 1 + 2^-53 lies halfway between 1 and 1 + 2^-52: the even neighbour is 1
    assert oracle.daxpy(1.0, np.array([2.0 ** -53]), np.array([1.0]))[0] == 1.0
    # (1 + 2^-52) + 2^-53 is halfway to 1 + 2^-51, which is even
    got = oracle.daxpy(1.0, np.array([2.0 ** -53]), np.array([1.0 + 2.0 ** -52]))
    assert got[0] == 1.0 + 2.0 ** -51
    # just above the tie rounds up
    got = oracle.daxpy(1.0 + 2.0 ** -52, np.array([2.0 ** -53]), np.array([1.0]))
    assert got[0] == 1.0 + 2.0 ** -52


def test_subnormal_results_are_exact():
    x = np.array([2.0 ** -1070, 3.0 * 2.0 ** -1074, 2.0 ** -1000])
    y = np.array([2.0 ** -1073, -(2.0 ** -1074), -(2.0 ** -1000)])
    got = oracle.daxpy(0.5, x, y)
    assert np.array_equal(got, oracle.exact_axpy(0.5, x, y))
    assert got[0] == 2.0 ** -1071 + 2.0 ** -1073


def test_special_values_propagate():
    inf, nan = np.inf, np.nan
    x = np.array([inf, inf, 1.0, nan, 2.0])
    y = np.array([1.0, inf, nan, 0.0, -inf])
    got = oracle.daxpy(-1.0, x, y)
    assert got[0] == -inf and np.isnan(got[1]) and np.isnan(got[2]) and np.isnan(got[3])
    assert got[4] == -inf


def test_quick_return_alpha_zero_and_empty():
    """alpha == 0 reads nothing: NaN/Inf in x leave y as it was."""
    y = synth.uniform_pm1(72, 0, 50)
    assert np.array_equal(oracle.daxpy(0.0, np.full(50, np.nan), y), y)
    assert np.array_equal(oracle.daxpy(2.0, np.ones(50), y, n=0), y)


def test_increments_touch_only_their_elements():
    n = 37
    x = synth.uniform_pm1(73, 0, 3 * n)
    y = synth.uniform_pm1(73, 1, 2 * n)
    got = oracle.daxpy(1.25, x, y, n=n, incx=3, incy=2)
    assert np.array_equal(got[0::2], oracle.exact_axpy(1.25, x[0::3], y[0::2]))
    assert np.array_equal(got[1::2], y[1::2])


def test_small_integers_and_closed_forms():
    x = synth.small_int_matrix(74, 0, 1, 1000)[0]
    y = synth.small_int_matrix(74, 1, 1, 1000)[0]
    assert np.array_equal(oracle.daxpy(3.0, x, y), 3.0 * x + y)
    assert np.array_equal(oracle.daxpy(-1.0, y, y), np.zeros(1000))
    assert np.array_equal(oracle.daxpy(1.0, x, np.zeros(1000)), x)


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.daxpy(1.0, np.ones(4), np.ones(4), n=3, incx=0)
    with pytest.raises(ValueError):
        oracle.daxpy(1.0, np.ones(4), np.ones(4), n=5)


# ------------------------------------------------------------ mutation tests
LINE = "y[i * incy] = fma(alpha, x[i * incx], y[i * incy]);"
MUTATIONS = {
    "unfused": "y[i * incy] = alpha * x[i * incx] + y[i * incy];",
    "dropped_y": "y[i * incy] = alpha * x[i * incx];",
    "sign_flip": "y[i * incy] = fma(alpha, x[i * incx], -y[i * incy]);",
    "wrong_increment": "y[i * incy] = fma(alpha, x[i * incy], y[i * incy]);",
}


def _pin_suite(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    f = lib.oracle_daxpy
    f.argtypes = [ctypes.c_int64, ctypes.c_double, dp, ctypes.c_int64, dp, ctypes.c_int64]

    def run(alpha, x, y, incx=1, incy=1):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.array(y, dtype=np.float64, copy=True)
        n = min((x.size + incx - 1) // incx, (out.size + incy - 1) // incy)
        f(n, alpha, x.ctypes.data_as(dp), incx, out.ctypes.data_as(dp), incy)
        return out

    ok = True
    x = synth.exp_spread(75, 0, 1, 200, -30, 30)
    y = synth.exp_spread(75, 2, 3, 200, -30, 30)
    ok &= bool(np.array_equal(run(0.75, x, y), oracle.exact_axpy(0.75, x, y)))
    a = 1.0 + 2.0 ** -30
    ok &= bool(run(a, [a], [-(1.0 + 2.0 ** -29)])[0] == 2.0 ** -60)
    xs = synth.uniform_pm1(75, 4, 60)
    ys = synth.uniform_pm1(75, 5, 40)
    got = run(1.5, xs, ys, incx=3, incy=2)
    ok &= bool(np.array_equal(got[0::2], oracle.exact_axpy(1.5, xs[0::3], ys[0::2])))
    return ok


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistakes(name, tmp_path):
    from oracle import build as ob
    src = open(ob.SRC).read()
    assert LINE in src
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(LINE, MUTATIONS[name]))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", *ob.CFLAGS, str(mutated), "-o", str(so), "-lm"], check=True)
    assert not _pin_suite(ctypes.CDLL(str(so))), name


def test_unmutated_oracle_passes_pin_suite():
    assert _pin_suite(ctypes.CDLL(oracle.LIB_PATH))
