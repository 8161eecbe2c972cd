"""Split-precision GEMM written out plainly (numpy), for testing only.

The paper computes DGEMM natively in FP64.  The split-precision form rebuilds
the FP64 product from exact low-precision pieces (an error-free splitting in
the style of Ozaki, Ogita, Oishi and Rump, "Error-free transformations of
matrix multiplication by using fast routines of matrix multiplication and its
applications", Numer. Algorithms 59, 2012), with integer slices so that the
slice products are exact on INT8 (INT32 accumulation) or BF16 (FP32
accumulation) matrix units.  The steps, in order:

1. Scale.  E_i = exponent e of frexp(max_p |A[i,p]|), so max |A[i,:]| < 2^E_i;
   F_j likewise for column j of B.  An all-zero row/column gets exponent 0.
2. Slice.  r_0 = A[i,p] * 2^-E_i lies in (-1, 1).  For t = 1..s:
   x = r_{t-1} * 2^b, A_t = trunc(x), r_t = x - A_t.  Every step is exact, so
   A[i,p] = 2^E_i * (sum_t A_t 2^(-b t) + r_s 2^(-b s)) with |A_t| < 2^b.
   b = 7 for INT8 slices ([-127, 127]), b = 8 for BF16 slices ([-255, 255],
   integers a BF16 holds exactly).  B is sliced the same way per column.
3. Products.  For each diagonal d = 2..s+1:  P_d = sum_{p+q=d} A_p B_q,
   pairs with 1 <= p, q <= s (the triangle p + q <= s + 1 is kept; the
   dropped terms are below 2^(-b(s+1)) relative to the row/column scales).
   P_d is an exact integer matrix.
4. Recombine.  acc = sum_{d=2}^{s+1} P_d * 2^(-b d), added in FP64 in
   increasing d;  C <- alpha * 2^(E_i + F_j) * acc + beta * C.

Step 3 is evaluated here with float64 matrix products of integer matrices:
every partial sum is an integer bounded by s * k * (2^b - 1)^2 < 2^53 (checked),
so any summation order returns the exact integer.
"""

from __future__ import annotations

import numpy as np

SPLIT_BITS = {"i8": 7, "bf16": 8}


def split_scales(X: np.ndarray, axis: int) -> np.ndarray:
    """Per-row (axis=1) or per-column (axis=0) exponents E with max|x| < 2^E."""
    X = np.asarray(X, dtype=np.float64)
    mx = np.max(np.abs(X), axis=axis) if X.shape[axis] > 0 else np.zeros(X.shape[1 - axis])
    _, e = np.frexp(mx)
    e = np.where(mx == 0.0, 0, e)
    return e.astype(np.int32)


def split_slices(X: np.ndarray, exps: np.ndarray, axis: int, s: int, bits: int):
    """Integer slices (as int32 array of shape (s,) + X.shape) and the
    remainder r_s, following step 2 of the module docstring.  ``exps`` are
    per-row exponents when axis == 1 and per-column when axis == 0."""
    X = np.asarray(X, dtype=np.float64)
    e = exps[:, None] if axis == 1 else exps[None, :]
    r = np.ldexp(X, -e.astype(np.int32))
    out = np.empty((s,) + X.shape, dtype=np.int32)
    for t in range(s):
        x = np.ldexp(r, bits)
        q = np.trunc(x)
        out[t] = q.astype(np.int32)
        r = x - q
    return out, r


def split_reconstruct(slices: np.ndarray, exps: np.ndarray, axis: int, bits: int) -> np.ndarray:
    """2^E * sum_t slice_t * 2^(-bits*t), accumulated smallest term first."""
    s = slices.shape[0]
    acc = np.zeros(slices.shape[1:], dtype=np.float64)
    for t in range(s, 0, -1):
        acc = acc + np.ldexp(slices[t - 1].astype(np.float64), -bits * t)
    e = exps[:, None] if axis == 1 else exps[None, :]
    return np.ldexp(acc, e.astype(np.int32))


def split_products(As: np.ndarray, Bs: np.ndarray, bits: int):
    """Exact diagonal products {d: P_d} for d = 2..s+1 (float64 holding integers)."""
    s = As.shape[0]
    k = As.shape[2]
    bound = s * k * (2 ** bits - 1) ** 2
    if bound >= 2 ** 53:
        raise ValueError("slice products would not be exact in float64")
    out = {}
    for d in range(2, s + 2):
        P = np.zeros((As.shape[1], Bs.shape[2]))
        for p in range(max(1, d - s), min(s, d - 1) + 1):
            q = d - p
            P += As[p - 1].astype(np.float64) @ Bs[q - 1].astype(np.float64)
        out[d] = P
    return out


def split_gemm(alpha: float, A, B, beta: float, C, s: int, kind: str = "i8") -> np.ndarray:
    """alpha * (split-precision approximation of A@B) + beta * C."""
    bits = SPLIT_BITS[kind]
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    E = split_scales(A, axis=1)
    F = split_scales(B, axis=0)
    As, _ = split_slices(A, E, 1, s, bits)
    Bs, _ = split_slices(B, F, 0, s, bits)
    P = split_products(As, Bs, bits)
    acc = np.zeros((A.shape[0], B.shape[1]))
    for d in range(2, s + 2):
        acc = acc + np.ldexp(P[d], -bits * d)
    prod = np.ldexp(acc, (E[:, None] + F[None, :]).astype(np.int32))
    out = alpha * prod
    if beta != 0.0:
        out = out + beta * np.asarray(C, dtype=np.float64)
    return out
