"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module generates numbers and nothing else: it holds none of the GEMM
arithmetic, imports neither the oracle nor the HIP library, and both of those
only ever see the arrays it returns.

Generator: counter-based SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  For a (seed, stream) pair the
key is the SplitMix64 finaliser applied to ``seed + GOLDEN*(stream+1)``; the
value at counter ``idx`` is the finaliser applied to ``key + GOLDEN*(idx+1)``,
i.e. the (idx+1)-th output of a SplitMix64 sequence started at ``key``.  Every
element therefore depends only on (seed, stream, idx), so any sub-block of a
matrix can be regenerated on its own and the numpy (host) and torch (device)
versions below give identical bits.

Matrix element (i, j) of a rows x cols matrix uses ``idx = i*cols + j``
(independent of the leading dimension), so a matrix stored with padding has the
same logical values as a dense one.

Workload recipes (the paper fills square dense matrices with random values
in [0, 10], Section 4.2; the configurations here use [-1, 1) instead and the
paper's range is kept as an extra case):
  * ``uniform_pm1``: x = 2u - 1 in [-1, 1), u = top 53 bits * 2^-53 (exact).
  * ``uniform_0_10``: 10u in [0, 10).
  * ``exp_spread``: (2u - 1) * 2^e with integer e uniform in [emin, emax],
    e taken from a second stream as floor(hi32 * (emax-emin+1) / 2^32) + emin.
  * ``log_uniform_int``: floor(exp(ln lo + u (ln(hi+1) - ln lo))) clamped to
    [lo, hi] (host only).
  * ``poisson_gaps``: -ln(1 - u) / rate (host only).
"""

from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB

# Stream ids: one independent sequence per role.
STREAM_A = 0
STREAM_B = 1
STREAM_C = 2
STREAM_EXP_A = 3
STREAM_EXP_B = 4
STREAM_SIZES = 5
STREAM_ARRIVALS = 6
STREAM_MIX = 7

BASE_SEED = 160208477


def config_seed(cfg: int, rep: int = 0) -> int:
    """Seed of repetition ``rep`` of workload configuration ``cfg`` (1-based)."""
    return BASE_SEED + 1000 * cfg + rep


_M64 = (1 << 64) - 1


def _mix_py(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * MIX1) & _M64
    z = ((z ^ (z >> 27)) * MIX2) & _M64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    return _mix_py(seed + GOLDEN * (stream + 1))


def bits_scalar(seed: int, stream: int, idx: int) -> int:
    """Reference scalar definition (pure Python ints) of one 64-bit output."""
    return _mix_py(stream_key(seed, stream) + GOLDEN * (idx + 1))


# ---------------------------------------------------------------- numpy (host)
def _bits_np(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    key = np.uint64(stream_key(seed, stream))
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = key + idx * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        z = z ^ (z >> np.uint64(31))
    return z


def _u53_to_pm1_np(z: np.ndarray) -> np.ndarray:
    u53 = (z >> np.uint64(11)).astype(np.int64)
    return (u53 - (1 << 52)).astype(np.float64) * 2.0 ** -52


def _u53_to_unit_np(z: np.ndarray) -> np.ndarray:
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


# ------------------------------------------------------------- torch (device)
def _bits_torch(seed: int, stream: int, start: int, count: int, device):
    import torch

    def s64(v: int) -> int:  # reinterpret an unsigned 64-bit constant as int64
        v &= _M64
        return v - (1 << 64) if v >= (1 << 63) else v

    def lsr(z, s):  # logical shift right on int64
        return (z >> s) & ((1 << (64 - s)) - 1)

    idx = torch.arange(start + 1, start + 1 + count, dtype=torch.int64, device=device)
    z = idx * s64(GOLDEN) + s64(stream_key(seed, stream))
    z = (z ^ lsr(z, 30)) * s64(MIX1)
    z = (z ^ lsr(z, 27)) * s64(MIX2)
    z = z ^ lsr(z, 31)
    return z


def _is_host(device) -> bool:
    return device is None or str(device) == "numpy"


# ------------------------------------------------------------------ public API
def uniform_pm1(seed: int, stream: int, count: int, start: int = 0, device=None):
    """``count`` values 2u-1 in [-1, 1); numpy array if ``device`` is None,
    else a float64 torch tensor on ``device``."""
    if _is_host(device):
        return _u53_to_pm1_np(_bits_np(seed, stream, start, count))
    z = _bits_torch(seed, stream, start, count, device)
    u53 = (z >> 11) & ((1 << 53) - 1)
    return (u53 - (1 << 52)).double() * 2.0 ** -52


def uniform_unit(seed: int, stream: int, count: int, start: int = 0):
    """``count`` values u in [0, 1) (host)."""
    return _u53_to_unit_np(_bits_np(seed, stream, start, count))


def uniform_0_10(seed: int, stream: int, count: int, start: int = 0):
    """The paper's fill range: 10u in [0, 10) (host)."""
    return 10.0 * uniform_unit(seed, stream, count, start)


def exponents(seed: int, stream: int, count: int, emin: int, emax: int,
              start: int = 0, device=None):
    """Integers uniform in [emin, emax] from the high 32 bits of each output."""
    span = emax - emin + 1
    if _is_host(device):
        z = _bits_np(seed, stream, start, count)
        hi = (z >> np.uint64(32)).astype(np.int64)
        return (hi * span >> 32) + emin
    z = _bits_torch(seed, stream, start, count, device)
    hi = (z >> 32) & 0xFFFFFFFF
    return ((hi * span) >> 32) + emin


def exp_spread(seed: int, stream_val: int, stream_exp: int, count: int,
               emin: int = -20, emax: int = 20, start: int = 0, device=None):
    """Values (2u-1) * 2^e, e uniform in [emin, emax] (exact products)."""
    x = uniform_pm1(seed, stream_val, count, start, device)
    e = exponents(seed, stream_exp, count, emin, emax, start, device)
    if _is_host(device):
        return np.ldexp(x, e.astype(np.int32))
    import torch
    return torch.ldexp(x, e.double())


def matrix(seed: int, stream: int, rows: int, cols: int, kind: str = "pm1",
           device=None, stream_exp: int | None = None):
    """Dense row-major rows x cols float64 matrix; element (i, j) uses counter
    i*cols + j.  ``kind``: 'pm1' (U[-1,1)), 'paper' (U[0,10)) or 'spread'
    ((2u-1)*2^e, e in [-20, 20], exponents from ``stream_exp``)."""
    count = rows * cols
    if kind == "pm1":
        v = uniform_pm1(seed, stream, count, device=device)
    elif kind == "paper":
        if not _is_host(device):
            raise ValueError("the [0,10) fill is generated on the host")
        v = uniform_0_10(seed, stream, count)
    elif kind == "spread":
        if stream_exp is None:
            stream_exp = {STREAM_A: STREAM_EXP_A, STREAM_B: STREAM_EXP_B}.get(stream, stream + 16)
        v = exp_spread(seed, stream, stream_exp, count, device=device)
    else:
        raise ValueError(f"unknown kind {kind!r}")
    return v.reshape(rows, cols)


def small_int_matrix(seed: int, stream: int, rows: int, cols: int, lo: int = -8, hi: int = 8):
    """Integers uniform in [lo, hi] as float64 (host)."""
    e = exponents(seed, stream, rows * cols, lo, hi)
    return e.astype(np.float64).reshape(rows, cols)


def log_uniform_int(seed: int, stream: int, count: int, lo: int, hi: int, start: int = 0):
    """Log-uniform integers in [lo, hi] (host)."""
    u = uniform_unit(seed, stream, count, start)
    x = np.floor(np.exp(np.log(lo) + u * (np.log(hi + 1) - np.log(lo))))
    return np.clip(x, lo, hi).astype(np.int64)


def poisson_gaps(seed: int, stream: int, count: int, rate: float, start: int = 0):
    """Exponential inter-arrival gaps in seconds for a Poisson process."""
    u = uniform_unit(seed, stream, count, start)
    return -np.log1p(-u) / rate


def batch_shapes(seed: int, count: int, lo: int = 16, hi: int = 512):
    """(count, 3) int64 array of (m, n, k), each log-uniform in [lo, hi]
    (independent draws from the sizes stream)."""
    v = log_uniform_int(seed, STREAM_SIZES, 3 * count, lo, hi)
    return v.reshape(count, 3)


def flat_uniform(seed: int, stream: int, count: int, device=None):
    """One long U[-1,1) vector (batched operands are carved out of it)."""
    return uniform_pm1(seed, stream, count, device=device)
