"""Pins for the oracle's reductions and AXPY body (CPU only).

Each check ties the oracle to something it does not compute itself:
closed forms of integer sums, Python's arbitrary-precision integers taken
modulo 2^w, Shewchuk's exactly rounded ``math.fsum``, exact rational
arithmetic for the fused multiply-add, planted extremes, and special cases
where plain FP32 summation provably fails.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _wrap(v, bits):
    v &= (1 << bits) - 1
    return v - (1 << bits) if v >> (bits - 1) else v


# ---------------------------------------------------------------- integers

@pytest.mark.parametrize("dt,bits", [(np.int32, 32), (np.int64, 64)])
def test_int_sum_closed_forms(dt, bits):
    for n in (0, 1, 2, 1000, 65537):
        a = np.arange(n, dtype=dt)
        assert oracle.reduce_int(a, "sum") == _wrap(n * (n - 1) // 2, bits)
        c = np.full(n, -7, dtype=dt)
        assert oracle.reduce_int(c, "sum", 5) == _wrap(5 - 7 * n, bits)


def test_int32_sum_wraps_to_zero():
    # 2^20 copies of 2^12 = 2^32 == 0 mod 2^32
    a = np.full(1 << 20, 1 << 12, dtype=np.int32)
    assert oracle.reduce_int(a, "sum") == 0
    # and one more element shows the wrap is two's complement
    b = np.concatenate([a, np.array([-1], dtype=np.int32)])
    assert oracle.reduce_int(b, "sum") == -1


def test_int64_sum_wraps():
    a = np.array([2**62, 2**62, 2**62, 2**62, 5], dtype=np.int64)
    assert oracle.reduce_int(a, "sum") == 5


@pytest.mark.parametrize("dt,bits", [(np.int32, 32), (np.int64, 64)])
def test_int_random_vs_bigint(dt, bits):
    g = np.random.Generator(np.random.PCG64(11))
    info = np.iinfo(dt)
    a = g.integers(info.min, info.max, size=5000, endpoint=True, dtype=dt)
    x0 = int(a[17])
    assert oracle.reduce_int(a, "sum", x0) == _wrap(x0 + sum(int(v) for v in a), bits)
    assert oracle.reduce_int(a, "max", info.min) == max(int(v) for v in a)
    assert oracle.reduce_int(a, "min", info.max) == min(int(v) for v in a)


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_int_max_min_permutation(dt):
    g = np.random.Generator(np.random.PCG64(3))
    n = 10007
    p = g.permutation(n).astype(dt)
    assert oracle.reduce_int(p, "max", np.iinfo(dt).min) == n - 1
    assert oracle.reduce_int(p, "min", np.iinfo(dt).max) == 0
    # x_orig participates in the fold
    assert oracle.reduce_int(p, "max", n + 5) == n + 5
    assert oracle.reduce_int(p, "min", -3) == -3
    # signed comparison, not unsigned
    assert oracle.reduce_int(np.array([-1, 1], dtype=dt), "max", np.iinfo(dt).min) == 1


# ---------------------------------------------------------------- floating

@pytest.mark.parametrize("n", [1, 10, 1000, 1 << 16, 1 << 22])
def test_fp32_sum_vs_fsum(n):
    g = np.random.Generator(np.random.PCG64(n))
    a = g.standard_normal(n, dtype=np.float32)
    exact = math.fsum(a.astype(np.float64).tolist() + [0.25])
    got, sabs = oracle.reduce_fp(a, "sum", 0.25, want_abs=True)
    assert abs(got - exact) <= 4 * 2**-53 * abs(exact) + 1e-300
    assert sabs == pytest.approx(math.fsum(np.abs(a.astype(np.float64)).tolist()), rel=1e-14)


def test_fp64_sum_vs_fsum_ill_conditioned():
    g = np.random.Generator(np.random.PCG64(5))
    base = g.standard_normal(20000) * 1e10
    a = np.concatenate([base, -base, g.standard_normal(100)])
    g.shuffle(a)
    exact = math.fsum(a.tolist())
    assert abs(oracle.reduce_fp(a, "sum") - exact) <= 4 * 2**-53 * abs(exact)


def test_fp32_all_ones_beyond_2pow24():
    n = (1 << 24) + 1000
    a = np.ones(n, dtype=np.float32)
    assert oracle.reduce_fp(a, "sum") == float(n)
    # plain sequential fp32 summation gets stuck at 2^24
    assert np.float32(1 << 24) + np.float32(1) == np.float32(1 << 24)


def test_fp32_big_then_many_ones():
    a = np.concatenate([np.array([1e8], dtype=np.float32), np.ones(1 << 20, dtype=np.float32)])
    assert oracle.reduce_fp(a, "sum") == float(np.float32(1e8)) + (1 << 20)


def test_bf16_widening_exact():
    g = np.random.Generator(np.random.PCG64(9))
    f = g.standard_normal(4096, dtype=np.float32)
    bits = (f.view(np.uint32) >> 16).astype(np.uint16)      # truncation: any bf16 pattern
    wid = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert oracle.reduce_fp(bits, "sum", bf16=True) == pytest.approx(math.fsum(wid.tolist()), rel=1e-15, abs=1e-300)
    assert oracle.reduce_fp(bits, "max", -np.inf, bf16=True) == wid.max()
    assert oracle.reduce_fp(bits, "min", np.inf, bf16=True) == wid.min()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_fp_planted_extremes(dt):
    g = np.random.Generator(np.random.PCG64(21))
    a = g.standard_normal(100003).astype(dt)
    a[77777] = 123.5
    a[4242] = -99.25
    assert oracle.reduce_fp(a, "max", -np.inf) == 123.5
    assert oracle.reduce_fp(a, "min", np.inf) == -99.25
    assert oracle.reduce_fp(a, "max", 500.0) == 500.0


def test_fp_max_min_nan_dropping_and_signed_zero():
    a = np.array([np.nan, -1.0, np.nan], dtype=np.float32)
    assert oracle.reduce_fp(a, "max", -np.inf) == -1.0
    assert oracle.reduce_fp(a, "min", np.inf) == -1.0
    z = np.array([-0.0, 0.0], dtype=np.float32)
    assert oracle.reduce_fp(z, "max", -np.inf) == 0.0
    assert oracle.reduce_fp(np.array([], dtype=np.float32), "max", -np.inf) == -np.inf


def test_empty_returns_x_orig():
    e32 = np.array([], dtype=np.int32)
    assert oracle.reduce_int(e32, "sum", 42) == 42
    assert oracle.reduce_fp(np.array([], dtype=np.float32), "sum", 1.5) == 1.5


# ---------------------------------------------------------------- AXPY

def _round_to_f32(q: Fraction) -> np.float32:
    """Exact round-to-nearest-even of a rational to binary32."""
    f = np.float32(float(q))           # within one ulp of the answer
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - q),
                                     int(np.array(c, dtype=np.float32).view(np.uint32)) & 1))
    return np.float32(best)


def test_axpy_fma_single_rounding_exact():
    g = np.random.Generator(np.random.PCG64(4))
    n = 3000
    x = g.standard_normal(n, dtype=np.float32)
    y = g.standard_normal(n, dtype=np.float32)
    # include cancellation-heavy cases where fma and mul+add differ
    x[:100] = np.float32(1.0) + np.float32(2.0**-12) * np.arange(100, dtype=np.float32)
    y[:100] = -np.float32(0.7) * x[:100]
    a = 0.7
    ynew, s = oracle.axpy_sum(a, x, y, 0.0)
    af = Fraction(float(np.float32(a)))
    want = np.array([_round_to_f32(af * Fraction(float(xi)) + Fraction(float(yi)))
                     for xi, yi in zip(x, y)], dtype=np.float32)
    assert np.array_equal(ynew.view(np.uint32), want.view(np.uint32))
    assert s == pytest.approx(math.fsum(want.astype(np.float64).tolist()), rel=1e-15, abs=1e-300)
    # the separately rounded product differs somewhere: the test would catch mul+add
    sep = (np.float32(a) * x + y).astype(np.float32)
    assert not np.array_equal(sep, want)
