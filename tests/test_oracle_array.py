"""Pins for the oracle's array-section reduction (CPU only): column folds of a
row-major block checked against closed forms and Shewchuk's math.fsum."""
import math

import numpy as np

import oracle


def test_int_columns_closed_form():
    R, m = 1001, 37
    a = (np.arange(R, dtype=np.int64)[:, None] * m + np.arange(m, dtype=np.int64)[None, :])
    s = oracle.reduce_array(a, "sum", [0] * m)
    assert s == [m * R * (R - 1) // 2 + j * R for j in range(m)]
    assert oracle.reduce_array(a, "max", [-(2**63)] * m) == [(R - 1) * m + j for j in range(m)]
    assert oracle.reduce_array(a, "min", [2**63 - 1] * m) == list(range(m))
    # x_orig takes part
    assert oracle.reduce_array(a[:, :2], "sum", [5, -5]) == [m * R * (R - 1) // 2 + 5, m * R * (R - 1) // 2 + R - 5]


def test_int32_columns_wrap():
    a = np.full((1 << 12, 3), 1 << 20, dtype=np.int32)   # 2^32 per column == 0
    a[0, 1] += 1
    assert oracle.reduce_array(a, "sum", [0, 0, 7]) == [0, 1, 7]


def test_fp_columns_vs_fsum():
    g = np.random.Generator(np.random.PCG64(2))
    a = g.standard_normal((5000, 9)).astype(np.float32)
    got = oracle.reduce_array(a, "sum", [0.0] * 9)
    for j in range(9):
        ref = math.fsum(a[:, j].astype(np.float64).tolist())
        assert abs(got[j] - ref) <= 4 * 2**-53 * abs(ref)


def test_single_row_and_column():
    a = np.array([[3, -4, 5]], dtype=np.int64)
    assert oracle.reduce_array(a, "sum", [1, 1, 1]) == [4, -3, 6]
    b = np.array([[1.5], [2.5], [-1.0]], dtype=np.float32)
    assert oracle.reduce_array(b, "sum", [0.0]) == [3.0]
