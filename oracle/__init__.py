"""CPU oracle for C <- alpha*A*B + beta*C and for the split-precision form.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the bench's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything here, and nothing here imports the product package.

Contents
  dgemm(...)            compensated (Dot2) FP64 oracle in C, see mg_oracle.c.
                        Follows the problem statement of Section 4.2 (DGEMM
                        computes C <- alpha A B + beta C).
  dgemm_sampled(...)    the same on a subset of output rows and columns.
  exact_gemm(...)       exact rational evaluation (Python fractions) rounded
                        once to the nearest double; for tiny cases only.
  rel_fro_err(...)      ||X - R||_F / ||R||_F (absolute norm if R == 0).
  daxpy(...)            y <- alpha x + y (Section 4.1), each element rounded
                        once (C, fma); exact_axpy(...) the rational form.
  split_*(...)          the split-precision method written out plainly in
                        numpy (not part of the paper; the method is the
                        Ozaki-style error-free splitting described in the
                        module docstring of ``split``).

The split-precision stages are exact integer work, so their pins are exact
(reconstruction identities, integer products); the final FP64 result is
compared to ``dgemm`` (the exact product) at the 1e-12 bar.
"""

from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

from .split import (split_scales, split_slices, split_reconstruct,  # noqa: F401
                    split_products, split_gemm, SPLIT_BITS)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmg_oracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_dgemm.argtypes = [i64, i64, i64, ctypes.c_double, dp, i64, dp, i64,
                                     ctypes.c_double, dp, i64]
        lib.oracle_dgemm.restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_daxpy.argtypes = [i64, ctypes.c_double, dp, i64, dp, i64]
        lib.oracle_daxpy.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return _load().oracle_threads()


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def dgemm(alpha: float, A: np.ndarray | None, B: np.ndarray | None, beta: float,
          C: np.ndarray | None, m: int | None = None, n: int | None = None,
          k: int | None = None) -> np.ndarray:
    """Return alpha*A@B + beta*C (new float64 array) with compensated sums.

    A is m x k, B is k x n, C is m x n (C may be None when beta == 0; A and B
    may be None when k == 0 or alpha == 0).  Inputs are converted to
    contiguous float64 (FP32 inputs are widened exactly)."""
    if A is not None:
        A = np.ascontiguousarray(A, dtype=np.float64)
        m = A.shape[0] if m is None else m
        k = A.shape[1] if k is None else k
    if B is not None:
        B = np.ascontiguousarray(B, dtype=np.float64)
        k = B.shape[0] if k is None else k
        n = B.shape[1] if n is None else n
    if C is not None:
        out = np.array(C, dtype=np.float64, order="C", copy=True)
        m, n = out.shape
    else:
        out = np.zeros((m, n), dtype=np.float64)
        if beta != 0.0:
            raise ValueError("beta != 0 needs C")
    if A is not None and A.shape != (m, k):
        raise ValueError("A shape mismatch")
    if B is not None and B.shape != (k, n):
        raise ValueError("B shape mismatch")
    if m == 0 or n == 0:
        return out
    dummy = np.zeros(1)
    a = A if A is not None and A.size else dummy
    b = B if B is not None and B.size else dummy
    rc = _load().oracle_dgemm(m, n, k, float(alpha), _ptr(a), max(k, 1), _ptr(b), max(n, 1),
                              float(beta), _ptr(out), n)
    if rc != 0:
        raise RuntimeError(f"oracle_dgemm failed with {rc}")
    return out


def dgemm_sampled(alpha, A, B, beta, C, rows, cols) -> np.ndarray:
    """Oracle values of the outputs (rows x cols) only: each needs one row of
    A and one column of B, so this is the definition applied element-wise."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    Cs = None if C is None else np.asarray(C)[np.ix_(rows, cols)]
    return dgemm(alpha, np.asarray(A)[rows, :], np.asarray(B)[:, cols], beta, Cs,
                 m=len(rows), n=len(cols), k=np.asarray(A).shape[1])


def exact_gemm(alpha, A, B, beta, C) -> np.ndarray:
    """Exact rational alpha*sum(a*b) + beta*c per element, rounded once to
    the nearest double (CPython's int/int division is correctly rounded).
    Pure Python; for tiny shapes only."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    al, be = Fraction(alpha), Fraction(beta)
    out = np.empty((m, n))
    for i in range(m):
        for j in range(n):
            acc = Fraction(0)
            for p in range(k):
                acc += Fraction(float(A[i, p])) * Fraction(float(B[p, j]))
            v = al * acc
            if beta != 0.0:
                v += be * Fraction(float(C[i, j]))
            out[i, j] = v.numerator / v.denominator
    return out


def daxpy(alpha: float, x: np.ndarray, y: np.ndarray, n: int | None = None, incx: int = 1,
          incy: int = 1) -> np.ndarray:
    """DAXPY (Section 4.1): return a copy of the flat buffer ``y`` with
    y[i*incy] <- alpha*x[i*incx] + y[i*incy] for i < n, each element the exact
    value rounded once (see mg_oracle.c).  n defaults to the most elements the
    buffers hold at these increments."""
    x = np.ascontiguousarray(np.ravel(x), dtype=np.float64)
    out = np.array(np.ravel(y), dtype=np.float64, copy=True)
    if n is None:
        n = min((x.size + incx - 1) // incx, (out.size + incy - 1) // incy)
    if n > 0 and ((n - 1) * incx >= x.size or (n - 1) * incy >= out.size):
        raise ValueError("buffers too short for n and the increments")
    rc = _load().oracle_daxpy(int(n), float(alpha), _ptr(x), int(incx), _ptr(out), int(incy))
    if rc != 0:
        raise ValueError(f"oracle_daxpy rejected its arguments ({rc})")
    return out


def exact_axpy(alpha: float, x, y) -> np.ndarray:
    """alpha*x[i] + y[i] evaluated exactly in rationals and rounded once to
    the nearest double (Python's Fraction -> float conversion rounds
    correctly, ties to even).  Finite inputs only; tiny cases."""
    a = Fraction(alpha)
    return np.array([float(a * Fraction(float(xi)) + Fraction(float(yi)))
                     for xi, yi in zip(np.ravel(x), np.ravel(y))], dtype=np.float64)


def rel_fro_err(X, R) -> float:
    """||X - R||_F / ||R||_F in float64 (||X - R||_F if R is all zero)."""
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    num = float(np.sqrt(np.sum(np.square(X - R))))
    den = float(np.sqrt(np.sum(np.square(R))))
    return num / den if den > 0 else num
