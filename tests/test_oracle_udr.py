"""Pins for the oracle's user-defined-reduction fold and sample moments, and
for the Python side of the test reductions (CPU only), against independent
computations:

* moments: closed forms (0..n-1 has mean (n-1)/2 and M2 = n (n^2 - 1) / 12; a
  constant sample has M2 = 0) and a hand-worked sample;
* the Welford fold equals the definitions within FP64 rounding, also when
  its result is combined pairwise from pieces (the combiner is the parallel
  formula of Chan et al.);
* STATS3, MINMAX, HIST16, SUMSQ folds equal numpy's vectorised counts, sums,
  min / max / argmin and bincount;
* an empty fold leaves x0 as it was; x0 takes part through the combiner.
"""
import math

import numpy as np
import pytest

import oracle
import synth
import udr_cases as U


def test_moments_closed_forms():
    for n in (1, 2, 10, 1001):
        c, mean, m2 = oracle.moments(np.arange(n, dtype=np.float64))
        assert c == n and mean == (n - 1) / 2 and math.isclose(m2, n * (n * n - 1) / 12, rel_tol=1e-15)
    assert oracle.moments(np.full(77, 3.25)) == (77.0, 3.25, 0.0)
    # 2, 4, 4, 4, 5, 5, 7, 9: mean 5, squared deviations 9+1+1+1+0+0+4+16 = 32
    assert oracle.moments(np.array([2, 4, 4, 4, 5, 5, 7, 9.0])) == (8.0, 5.0, 32.0)


def test_welford_fold_matches_definition():
    x = synth.f32_normal(20000, 5).astype(np.float64) * 3 + 100
    c, mean, m2 = oracle.moments(x)
    got = oracle.udr_fold(x, U.welford_init(), U.welford_init, U.welford_body, U.welford_combine)
    assert got[0] == c
    assert abs(got[1] - mean) <= 1e-13 * abs(mean)
    assert abs(got[2] - m2) <= 1e-11 * m2
    # pieces combined pairwise in a tree give the same moments
    parts = [oracle.udr_fold(x[k::7], U.welford_init(), U.welford_init, U.welford_body,
                             U.welford_combine) for k in range(7)]
    while len(parts) > 1:
        parts = [U.welford_combine(parts[j], parts[j + 1]) if j + 1 < len(parts) else parts[j]
                 for j in range(0, len(parts), 2)]
    assert parts[0][0] == c and abs(parts[0][1] - mean) <= 1e-13 * abs(mean)
    assert abs(parts[0][2] - m2) <= 1e-11 * m2


def test_exact_folds_match_numpy():
    v = synth.int32_uniform(5000, 8, lo=-(2 ** 31), hi=2 ** 31 - 1)
    got = oracle.udr_fold(v, (0, 0, 0), U.stats3_init, U.stats3_body, U.stats3_combine)
    cnt3 = int(np.count_nonzero(v.astype(np.int64) % 3 == 0))
    sq = int((v.astype(np.int64) * v.astype(np.int64)).astype(np.uint64).sum(dtype=np.uint64))
    idx = np.arange(1, v.size + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        hashes = (idx * np.uint64(U.GOLD)) ^ v.view(np.uint32).astype(np.uint64)
    assert got == (cnt3, sq, int(np.bitwise_xor.reduce(hashes)))

    f = synth.f64_normal(3000, 9)
    f[100] = f[2000] = -10.0                       # a tie for the minimum: first position
    got = oracle.udr_fold(f, U.minmax_init(), U.minmax_init, U.minmax_body, U.minmax_combine)
    assert got[:3] == (f.min(), f.max(), int(np.argmin(f))) and got[2] == 100

    k = synth.int64_uniform(4000, 10)
    got = oracle.udr_fold(k, U.hist16_init(), U.hist16_init, U.hist16_body, U.hist16_combine)
    assert list(got) == np.bincount((k & 15).astype(np.int64), minlength=16).tolist()

    s = synth.f32_normal(3000, 11).astype(np.float64)
    got = oracle.udr_fold(s, (0.0,), U.sumsq_init, U.sumsq_body, U.sumsq_combine)
    assert math.isclose(got[0], math.fsum(s * s), rel_tol=1e-13)


def test_x0_and_empty():
    x0 = (5, 7, 11)
    assert oracle.udr_fold([], x0, U.stats3_init, U.stats3_body, U.stats3_combine) == x0
    got = oracle.udr_fold([3, 4], x0, U.stats3_init, U.stats3_body, U.stats3_combine)
    assert got[:2] == (6, 7 + 9 + 16)


@pytest.mark.parametrize("name", sorted(U.FORMATS))
def test_pack_round_trip(name):
    init = getattr(U, name.lower() + "_init")()
    assert U.unpack(name, U.pack(name, init)) == tuple(init)
