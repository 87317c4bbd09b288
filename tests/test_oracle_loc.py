"""Pins for the oracle's maxloc / minloc (CPU only): numpy's first-occurrence
argmax / argmin and nanargmax / nanargmin, planted ties (the smaller position
wins), x_orig winning, losing and tying, NaN never winning, -0 == +0."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("dt", [np.int32, np.int64, np.float32, np.float64])
def test_matches_numpy_first_occurrence(dt):
    g = np.random.Generator(np.random.PCG64(4))
    for n in (1, 7, 1000, 100003):
        a = g.integers(-50, 50, n).astype(dt)          # many ties
        v, p = oracle.reduce_loc(a, "max", np.iinfo(np.int64).min if dt in (np.int32, np.int64) else -np.inf, -1)
        assert p == int(np.argmax(a)) and v == a[p]
        v, p = oracle.reduce_loc(a, "min", np.iinfo(np.int64).max if dt in (np.int32, np.int64) else np.inf, -1)
        assert p == int(np.argmin(a)) and v == a[p]


def test_x_orig_takes_part():
    a = np.array([3, 9, 9, 1], dtype=np.int32)
    assert oracle.reduce_loc(a, "max", 10, 42) == (10, 42)      # x_orig wins
    assert oracle.reduce_loc(a, "max", 5, 42) == (9, 1)         # loses
    assert oracle.reduce_loc(a, "max", 9, 0) == (9, 0)          # ties, smaller position
    assert oracle.reduce_loc(a, "max", 9, 5) == (9, 1)
    assert oracle.reduce_loc(a, "min", 1, 7) == (1, 3)
    assert oracle.reduce_loc(np.array([], dtype=np.int64), "min", 4, 2) == (4, 2)


def test_nan_and_signed_zero():
    a = np.array([np.nan, 2.0, np.nan, 5.0, 5.0, np.nan], dtype=np.float32)
    assert oracle.reduce_loc(a, "max", -np.inf, -1) == (5.0, 3) and np.nanargmax(a) == 3
    assert oracle.reduce_loc(a, "min", np.inf, -1) == (2.0, 1) and np.nanargmin(a) == 1
    assert oracle.reduce_loc(a, "max", np.nan, 99) == (5.0, 3)  # a NaN x_orig loses
    allnan = np.full(4, np.nan)
    assert oracle.reduce_loc(allnan, "max", -np.inf, -1) == (-np.inf, -1)
    z = np.array([0.0, -0.0], dtype=np.float64)
    v, p = oracle.reduce_loc(z, "min", np.inf, -1)
    assert p == 0 and v == 0.0
    v, p = oracle.reduce_loc(z[::-1].copy(), "max", -np.inf, -1)
    assert p == 0 and np.signbit(v)                              # -0 first: equal, smaller position


def test_bf16():
    bits = np.array([0x3F80, 0x4000, 0x4000, 0xC000], dtype=np.uint16)   # 1, 2, 2, -2
    assert oracle.reduce_loc(bits, "max", -np.inf, -1, bf16=True) == (2.0, 1)
    assert oracle.reduce_loc(bits, "min", np.inf, -1, bf16=True) == (-2.0, 3)
