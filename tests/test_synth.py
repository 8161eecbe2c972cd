"""The shared seeded input generator (no GPU)."""

import os

import numpy as np
import torch

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_published_sequence():
    want = [int(l, 16) for l in open(GOLDEN) if l.startswith("0x")]
    got = [synth._mix_py(synth.GOLDEN * (i + 1)) for i in range(len(want))]
    assert got == want


def test_numpy_and_torch_bits_agree():
    for seed, stream in [(0, 0), (7, 3), (synth.config_seed(3), synth.STREAM_B)]:
        a = synth.uniform_pm1(seed, stream, 5000, start=123)
        b = synth.uniform_pm1(seed, stream, 5000, start=123, device="cpu").numpy()
        assert np.array_equal(a, b)
        e = synth.exponents(seed, stream, 5000, -20, 20)
        f = synth.exponents(seed, stream, 5000, -20, 20, device="cpu").numpy()
        assert np.array_equal(e, f)
    s1 = synth.matrix(3, 0, 40, 50, kind="spread")
    s2 = synth.matrix(3, 0, 40, 50, kind="spread", device="cpu").numpy()
    assert np.array_equal(s1, s2)


def test_counter_based_subblocks():
    full = synth.uniform_pm1(9, 1, 1000)
    assert np.array_equal(full[400:600], synth.uniform_pm1(9, 1, 200, start=400))
    assert synth.bits_scalar(9, 1, 17) == int(synth._bits_np(9, 1, 17, 1)[0])


def test_ranges_and_exactness():
    x = synth.uniform_pm1(1, 0, 200000)
    assert x.min() >= -1.0 and x.max() < 1.0
    assert abs(x.mean()) < 0.01
    # values are k * 2^-52: exact multiples
    assert np.array_equal(np.ldexp(x, 52), np.trunc(np.ldexp(x, 52)))
    e = synth.exponents(1, 3, 200000, -20, 20)
    assert e.min() == -20 and e.max() == 20
    counts = np.bincount(e + 20)
    assert counts.min() > 0.9 * len(e) / 41
    s = synth.matrix(1, 0, 300, 300, kind="spread")
    assert np.abs(s).max() < 2.0 ** 20 and np.abs(s).min() > 0


def test_log_uniform_and_poisson():
    v = synth.log_uniform_int(1, synth.STREAM_SIZES, 100000, 16, 512)
    assert v.min() == 16 and v.max() == 512
    # log-uniform: about as many in [16,32) as in [256,512)
    lo = ((v >= 16) & (v < 32)).sum()
    hi = ((v >= 256) & (v < 512)).sum()
    assert 0.8 < lo / hi < 1.25
    g = synth.poisson_gaps(1, synth.STREAM_ARRIVALS, 100000, 2000.0)
    assert abs(g.mean() - 1 / 2000.0) < 0.02 / 2000.0


def test_torch_generator_keeps_dtype():
    t = synth.uniform_pm1(2, 0, 10, device="cpu")
    assert t.dtype == torch.float64
