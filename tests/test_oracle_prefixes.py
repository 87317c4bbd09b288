"""Pins for the oracle's prefix folds (CPU only): the sum / max / min of every
requested prefix, read out of one pass, against values the oracle does not
compute itself -- Python big-integer sums modulo 2^w, Shewchuk's exactly
rounded math.fsum (the FP64 Neumaier sum is within a few ulps of it at these
sizes), numpy's max / min of the prefix, and exact rational fused
multiply-adds rounded once to binary32 for the AXPY body.  Lengths arrive in
any order, repeated, including 0 and the whole array.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def _wrap(v, bits):
    v &= (1 << bits) - 1
    return v - (1 << bits) if v >> (bits - 1) else v


LENS = [5000, 0, 1, 4999, 17, 5000, 2048, 3]


@pytest.mark.parametrize("dt,bits", [(np.int32, 32), (np.int64, 64)])
def test_int_prefixes_vs_bigint(dt, bits):
    g = np.random.Generator(np.random.PCG64(21))
    info = np.iinfo(dt)
    a = g.integers(info.min, info.max, size=5000, endpoint=True, dtype=dt)
    py = [int(v) for v in a]
    sums = oracle.fold_prefixes(a, "sum", LENS)
    mx = oracle.fold_prefixes(a, "max", LENS)
    mn = oracle.fold_prefixes(a, "min", LENS)
    for k, L in enumerate(LENS):
        assert sums[k] == _wrap(sum(py[:L]), bits), L
        assert mx[k] == (max(py[:L]) if L else int(info.min)), L
        assert mn[k] == (min(py[:L]) if L else int(info.max)), L


def test_int32_prefix_sum_wraps_and_x_takes_part():
    a = np.full(1 << 20, 1 << 12, dtype=np.int32)          # 2^20 * 2^12 = 2^32 == 0
    assert oracle.fold_prefixes(a, "sum", [1 << 20, 1 << 19], x=9) == [9, _wrap(9 + 2**31, 32)]


@pytest.mark.parametrize("bf16", [False, True])
def test_fp_prefixes_vs_fsum(bf16):
    n = 20001
    if bf16:
        a = synth.bf16_normal(n, 22)
        vals = (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        a = synth.f32_normal(n, 22)
        vals = a.astype(np.float64)
    lens = [n, 0, 1, 7, 10000, 19999, n, 333]
    sums = oracle.fold_prefixes(a, "sum", lens, bf16=bf16)
    mx = oracle.fold_prefixes(a, "max", lens, bf16=bf16)
    mn = oracle.fold_prefixes(a, "min", lens, x=0.25, bf16=bf16)
    for k, L in enumerate(lens):
        exact = math.fsum(vals[:L])
        assert abs(sums[k] - exact) <= 4 * 2.0 ** -53 * max(math.fsum(np.abs(vals[:L])), 1e-300), L
        assert mx[k] == (float(vals[:L].max()) if L else -math.inf), L
        assert mn[k] == (min(0.25, float(vals[:L].min())) if L else 0.25), L


def test_fp_prefix_sum_where_fp32_loses_everything():
    # 1e8 followed by ones: plain fp32 accumulation never moves off 1e8
    a = np.concatenate([np.array([1e8], np.float32), np.ones(1 << 16, np.float32)])
    assert oracle.fold_prefixes(a, "sum", [1, 1 + (1 << 16), 1001]) == [1e8, 1e8 + (1 << 16), 1e8 + 1000]


def _round_to_f32(q: Fraction) -> np.float32:
    """Exact round-to-nearest-even of a rational to binary32."""
    f = np.float32(float(q))           # within one ulp of the answer
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - q),
                                     int(np.array(c, dtype=np.float32).view(np.uint32)) & 1))
    return np.float32(best)


def test_axpy_prefix_sums_vs_exact():
    n = 4001
    x = synth.f32_normal(n, 23)
    y = synth.f32_normal(n, 24)
    y_in = y.copy()
    lens = [n, 1, 0, 2000, 4000]
    y2, sums = oracle.axpy_prefix_sums(0.7, x, y, lens, s_orig=1.5)
    assert np.array_equal(y, y_in)                               # y itself untouched
    af = Fraction(float(np.float32(0.7)))
    want = np.array([_round_to_f32(af * Fraction(float(xi)) + Fraction(float(yi)))
                     for xi, yi in zip(x, y)], dtype=np.float32)
    assert np.array_equal(y2.view(np.uint32), want.view(np.uint32))
    yv = want.astype(np.float64)
    for k, L in enumerate(lens):
        exact = math.fsum([1.5] + list(yv[:L]))
        assert abs(sums[k] - exact) <= 4 * 2.0 ** -53 * (1.5 + math.fsum(np.abs(yv[:L]))), L


def test_prefix_bad_arguments():
    a = np.arange(10, dtype=np.int64)
    with pytest.raises(ValueError):
        oracle.fold_prefixes(a, "sum", [11])
    with pytest.raises(ValueError):
        oracle.fold_prefixes(a, "prod", [3])
