"""Pins for the oracle's remaining OpenMP reduction identifiers (CPU only):
* (product), & | ^ (bitwise), && || (logical).

Each is tied to something the oracle does not compute itself: closed forms,
Python's unbounded integers reduced modulo 2^w, numpy's bitwise reductions,
exact rational products (fractions) within the stated FP64 bound, and
hand-placed zeros / NaNs for the logical folds.
"""
import math
from fractions import Fraction
from functools import reduce

import numpy as np
import pytest

import oracle


def wrap(v, bits):
    v %= 1 << bits
    return v - (1 << bits) if v >= 1 << (bits - 1) else v


@pytest.mark.parametrize("dt,bits", [(np.int32, 32), (np.int64, 64)])
def test_integer_product_wraps(dt, bits):
    for k in (0, 1, 20, 21, 41, 1000):
        a = np.full(k, 3, dtype=dt)
        assert oracle.reduce_int(a, "prod", 1) == wrap(3 ** k, bits)
        assert oracle.reduce_int(a, "prod", 5) == wrap(5 * 3 ** k, bits)
    g = np.random.Generator(np.random.PCG64(1))
    a = g.integers(-7, 8, 5000).astype(dt)
    assert oracle.reduce_int(a, "prod", -3) == wrap(reduce(lambda p, v: p * int(v), a, -3), bits)
    a[1234] = 0
    assert oracle.reduce_int(a, "prod", 1) == 0


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_bitwise(dt):
    bits = 8 * np.dtype(dt).itemsize
    pw = np.array([1 << i for i in range(bits - 1)], dtype=dt)
    assert oracle.reduce_int(pw, "bor", 0) == (1 << (bits - 1)) - 1
    assert oracle.reduce_int(pw, "band", -1) == 0
    assert oracle.reduce_int(np.full(10, -1, dtype=dt), "band", -1) == -1
    assert oracle.reduce_int(np.array([77, 77], dtype=dt), "bxor", 0) == 0
    g = np.random.Generator(np.random.PCG64(2))
    info = np.iinfo(dt)
    a = g.integers(info.min, info.max, 10001, dtype=dt, endpoint=True)
    for op, ufunc, x in (("band", np.bitwise_and, -1), ("bor", np.bitwise_or, 0),
                         ("bxor", np.bitwise_xor, 0)):
        assert oracle.reduce_int(a, op, x) == int(ufunc.reduce(a))
    assert oracle.reduce_int(a, "bxor", 12345) == int(np.bitwise_xor.reduce(a)) ^ 12345


@pytest.mark.parametrize("dt", [np.int32, np.int64, np.float32, np.float64])
def test_logical(dt):
    fold = oracle.reduce_int if dt in (np.int32, np.int64) else oracle.reduce_fp
    a = np.arange(1, 1001).astype(dt)
    assert fold(a, "land", 1) == 1 and fold(a, "lor", 0) == 1
    assert fold(a, "land", 0) == 0            # x_orig takes part
    for pos in (0, 500, 999):
        b = a.copy()
        b[pos] = 0
        assert fold(b, "land", 1) == 0
    z = np.zeros(100, dtype=dt)
    assert fold(z, "lor", 0) == 0 and fold(z, "lor", 7) == 1
    z[37] = -3
    assert fold(z, "lor", 0) == 1
    assert fold(np.array([], dtype=dt), "land", 1) == 1
    assert fold(np.array([], dtype=dt), "lor", 0) == 0


def test_logical_floating_special_values():
    a = np.array([1.0, np.nan, 2.0], dtype=np.float32)        # NaN is not zero: true
    assert oracle.reduce_fp(a, "land", 1.0) == 1.0
    b = np.array([-0.0, 0.0], dtype=np.float64)                # both zeros are false
    assert oracle.reduce_fp(b, "lor", 0.0) == 0.0
    bf = np.array([0x3F80, 0x8000], dtype=np.uint16)           # bf16 1.0 and -0.0
    assert oracle.reduce_fp(bf, "land", 1.0, bf16=True) == 0.0
    assert oracle.reduce_fp(bf, "lor", 0.0, bf16=True) == 1.0


def test_floating_product_closed_forms():
    for k in (0, 1, 10, 100):
        assert oracle.reduce_fp(np.full(k, 2.0, dtype=np.float32), "prod", 1.0) == 2.0 ** k
        assert oracle.reduce_fp(np.full(k, 0.5, dtype=np.float64), "prod", 3.0) == 3.0 * 0.5 ** k
    bf2 = np.full(20, 0x4000, dtype=np.uint16)                 # bf16 2.0
    assert oracle.reduce_fp(bf2, "prod", 1.0, bf16=True) == 2.0 ** 20
    assert oracle.reduce_fp(np.array([1.0, 0.0, 5.0], dtype=np.float32), "prod", 1.0) == 0.0


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_floating_product_within_its_bound(dt):
    g = np.random.Generator(np.random.PCG64(3))
    for n in (10, 1000, 3000):
        a = (1.0 + 0.01 * g.standard_normal(n)).astype(dt)
        exact = reduce(lambda p, v: p * Fraction(float(v)), a, Fraction(1))
        got = oracle.reduce_fp(a, "prod", 1.0)
        assert abs(Fraction(got) - exact) <= (n + 1) * Fraction(1, 2 ** 53) * abs(exact)
        assert math.isclose(got, float(exact), rel_tol=1e-12)
