"""Pins for the oracle's histogram reduction (CPU only): numpy's bincount,
a hand-worked example, keys outside the bins, x_orig (the incoming
histogram) taking part, and int32 wrap of a count."""
import numpy as np

import oracle


def test_matches_bincount():
    g = np.random.Generator(np.random.PCG64(8))
    for bins in (1, 7, 256, 5000):
        keys = g.integers(0, bins, 100003).astype(np.int32)
        h, sk = oracle.histogram(keys, bins)
        assert sk == 0 and np.array_equal(h, np.bincount(keys, minlength=bins))


def test_worked_example_and_out_of_range():
    h, sk = oracle.histogram([2, 0, 2, 5, -1, 2, 3], 4, hist=[10, 0, 0, 1])
    assert h.tolist() == [11, 0, 3, 2] and sk == 2


def test_count_wraps():
    keys = np.zeros(10, dtype=np.int32)
    h, _ = oracle.histogram(keys, 1, hist=[2**31 - 5])
    assert h.tolist() == [-(2**31) + 5]
