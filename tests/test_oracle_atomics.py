"""Pins for the oracle's device atomics (CPU only).

Worked examples of the five operations the paper lists for the device
runtime (sec. 3.1): add, max (unsigned compare), exchange, cas, and inc with
its wrap-around definition { v = x; x = x >= e ? 0 : x + 1 }.  The values
below are derived by hand from those definitions.
"""
import numpy as np

import oracle


def test_inc_wraps_at_e():
    t, old, sk = oracle.atomic_serial("inc", [0], [0] * 10, [3] * 10)
    assert old.tolist() == [0, 1, 2, 3, 0, 1, 2, 3, 0, 1]
    assert t.tolist() == [2] and sk == 0
    # e = 0: every inc reads 0 and leaves 0 (a one-participant election)
    t, old, _ = oracle.atomic_serial("inc", [0], [0] * 4, [0] * 4)
    assert old.tolist() == [0, 0, 0, 0] and t.tolist() == [0]
    # a value already above e wraps to 0 on the first inc
    t, old, _ = oracle.atomic_serial("inc", [9], [0, 0], [3, 3])
    assert old.tolist() == [9, 0] and t.tolist() == [1]


def test_add_returns_prefix_and_wraps():
    t, old, _ = oracle.atomic_serial("add", [5], [0, 0, 0], [7, 7, 7])
    assert old.tolist() == [5, 12, 19] and t.tolist() == [26]
    t, old, _ = oracle.atomic_serial("add", [0xFFFFFFFF], [0], [2])
    assert old.tolist() == [0xFFFFFFFF] and t.tolist() == [1]


def test_max_is_unsigned():
    t, old, _ = oracle.atomic_serial("max", [0x80000000], [0, 0], [5, 0x90000000])
    assert old.tolist() == [0x80000000, 0x80000000] and t.tolist() == [0x90000000]
    t, _, _ = oracle.atomic_serial("max", [7], [0], [3])
    assert t.tolist() == [7]


def test_exchange_chain():
    t, old, _ = oracle.atomic_serial("exchange", [1], [0, 0, 0], [10, 20, 30])
    assert old.tolist() == [1, 10, 20] and t.tolist() == [30]


def test_cas_success_then_failure():
    t, old, _ = oracle.atomic_serial("cas", [4], [0, 0, 0], [4, 4, 8], [8, 9, 11])
    # first: 4 == 4 -> 8; second: 8 != 4 -> unchanged; third: 8 == 8 -> 11
    assert old.tolist() == [4, 8, 8] and t.tolist() == [11]


def test_independent_targets_and_out_of_range():
    t, old, sk = oracle.atomic_serial("add", [0, 100, 200], [2, 0, 7, 2], [1, 2, 3, 4])
    assert t.tolist() == [2, 100, 205]
    assert old.tolist() == [200, 0, 0xFFFFFFFF, 201] and sk == 1


def test_inc_election_any_arrival_order():
    # T participants each inc once with e = T - 1: the reads are 0..T-1, once each
    for T in (1, 2, 7, 64):
        t, old, _ = oracle.atomic_serial("inc", [0], [0] * T, [T - 1] * T)
        assert sorted(old.tolist()) == list(range(T)) and t.tolist() == [0]
