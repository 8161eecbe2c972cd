"""Parity of the DAXPY HIP kernels (mg_daxpy) with the CPU oracle, needs a GPU.

y <- alpha*x + y with every element one fused multiply-add: the bar is
bit-exact equality with the oracle (the exact value rounded once) on every
element, for lengths around the kernel's 16-byte pairs and 4 KB workgroup
spans, both 16-byte phases of x and y (vector path when they agree,
element-wise path when they differ), positive increments, y aliasing x, the
quick return and IEEE special values; the elements of y's buffer outside the
vector must keep their canaries.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mg = pytest.importorskip("paper_1602_08477_amd")

CANARY = 4242.0
LENGTHS = [1, 2, 3, 7, 255, 256, 257, 1023, 2048, 2049, 4097, 1_000_003, (1 << 22) + 5]


def device_vec(host, off, inc=1, pad=3):
    """Device buffer holding ``host`` at element offset ``off`` with increment
    ``inc`` (canaries everywhere else); returns (buffer, strided view)."""
    n = host.size
    size = off + (n - 1) * inc + 1 + pad if n else off + pad
    buf = torch.full((size,), CANARY, dtype=torch.float64, device="cuda")
    view = buf[off: off + (n - 1) * inc + 1: inc] if n else buf[off:off]
    if n:
        view.copy_(torch.from_numpy(host))
    return buf, view


def expected_buffer(buf_host, off, inc, n, alpha, x):
    y = buf_host[off: off + (n - 1) * inc + 1: inc]
    out = buf_host.copy()
    out[off: off + (n - 1) * inc + 1: inc] = oracle.daxpy(alpha, x, y)
    return out


@pytest.mark.parametrize("offs", [(0, 0), (1, 1), (0, 1), (1, 0)])
@pytest.mark.parametrize("n", LENGTHS)
def test_daxpy_bit_exact(n, offs):
    ox, oy = offs
    log(f"daxpy n={n} offsets={offs}")
    x = synth.exp_spread(80, 0, 1, n, -30, 30)
    y = synth.exp_spread(80, 2, 3, n, -30, 30)
    _, dx = device_vec(x, ox)
    ybuf, dy = device_vec(y, oy)
    before = ybuf.cpu().numpy()
    mg.daxpy(-1.375, dx, dy)
    torch.cuda.synchronize()
    assert np.array_equal(ybuf.cpu().numpy(), expected_buffer(before, oy, 1, n, -1.375, x))


@pytest.mark.parametrize("incs", [(2, 1), (1, 3), (3, 2), (5, 5)])
@pytest.mark.parametrize("n", [1, 100, 4099, 300_001])
def test_daxpy_increments(n, incs):
    incx, incy = incs
    x = synth.uniform_pm1(81, 0, n)
    y = synth.uniform_pm1(81, 1, n)
    _, dx = device_vec(x, 1, incx)
    ybuf, dy = device_vec(y, 0, incy)
    before = ybuf.cpu().numpy()
    mg.daxpy(0.625, dx, dy)
    torch.cuda.synchronize()
    assert np.array_equal(ybuf.cpu().numpy(), expected_buffer(before, 0, incy, n, 0.625, x))


@pytest.mark.parametrize("off", [0, 1])
def test_daxpy_y_is_x(off):
    n = 100_001
    x = synth.uniform_pm1(82, 0, n)
    buf, d = device_vec(x, off)
    mg.daxpy(3.0, d, d)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), oracle.daxpy(3.0, x, x))


def test_daxpy_quick_return_and_special_values():
    n = 1000
    y = synth.uniform_pm1(83, 0, n)
    ybuf, dy = device_vec(y, 0)
    _, dnan = device_vec(np.full(n, np.nan), 0)
    mg.daxpy(0.0, dnan, dy)                       # alpha == 0: x is not read
    mg.daxpy(2.0, dnan[:0], dy[:0])               # n == 0
    torch.cuda.synchronize()
    assert np.array_equal(dy.cpu().numpy(), y)
    xs = np.array([np.inf, np.inf, 1.0, np.nan, 2.0, 0.0, -0.0])
    ys = np.array([1.0, np.inf, np.nan, 0.0, -np.inf, -0.0, -0.0])
    _, dx = device_vec(xs, 0)
    _, dy2 = device_vec(ys, 0)
    mg.daxpy(-1.0, dx, dy2)
    torch.cuda.synchronize()
    got, ref = dy2.cpu().numpy(), oracle.daxpy(-1.0, xs, ys)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    fin = ~np.isnan(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.signbit(got[fin]), np.signbit(ref[fin]))


def test_daxpy_full_size_bit_exact():
    """The bench workload: n = 2^27 (1 GiB per vector), U[-1,1), alpha = 1.5,
    every element against the oracle."""
    n = 1 << 27
    log("daxpy full size")
    seed = synth.config_seed(3)
    dx = synth.uniform_pm1(seed, 0, n, device="cuda")
    dy = synth.uniform_pm1(seed, 1, n, device="cuda")
    x, y = dx.cpu().numpy(), dy.cpu().numpy()
    mg.daxpy(1.5, dx, dy)
    torch.cuda.synchronize()
    assert np.array_equal(dy.cpu().numpy(), oracle.daxpy(1.5, x, y))
