"""Pins for the oracle's static iteration map (CPU only).

The oracle enumerates the schedule (teams -> distribute chunks -> threads ->
chunks -> iterations).  These tests check it against things it does not
compute that way:

* an inverse closed form: the owner of iteration i derived directly from i
  (which team block / dealt chunk contains i, then which thread's);
* invariants the OpenMP static rules fix (every iteration exactly once,
  chunk sizes, balance, round-robin order, determinism);
* the hand-worked 2^20 x (1 team x 256 threads) example, default chunk and
  chunk 7 (tests/golden/static_map_c1.json).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "static_map_c1.json")


def _inv_balanced(i, m, p):
    """Which of p workers owns local index i of a balanced split of m (closed form)."""
    q, r = divmod(m, p)
    if i < r * (q + 1):
        return i // (q + 1)
    return r + (i - r * (q + 1)) // q


def _closed_form_owner(i, n, T, P, dc, c):
    # team and the bounds of the distribute chunk holding i
    if dc == 0:
        k = _inv_balanced(i, n, T)
        q, r = divmod(n, T)
        a = k * q + min(k, r)
        b = a + q + (1 if k < r else 0)
    else:
        j = i // dc
        k = j % T
        a, b = j * dc, min(n, (j + 1) * dc)
    m, li = b - a, i - a
    t = _inv_balanced(li, m, P) if c == 0 else (li // c) % P
    return k * P + t


TINY = [(n, T, P, dc, c)
        for n in (0, 1, 2, 3, 5, 8, 13, 17, 31, 64)
        for T in (1, 2, 3, 6)
        for P in (1, 2, 4, 9)
        for dc in (0, 1, 2, 5)
        for c in (0, 1, 2, 3, 7, 65)]


def test_closed_form_matches_enumeration_tiny():
    for n, T, P, dc, c in TINY:
        owner, count = oracle.iteration_map(n, T, P, dc, c)
        assert np.all(count == 1), (n, T, P, dc, c)
        want = [_closed_form_owner(i, n, T, P, dc, c) for i in range(n)]
        assert owner.tolist() == want, (n, T, P, dc, c)


def test_every_chunk_n_plus_one_exhaustive():
    # all chunk sizes 1..n+1 for a few shapes, including c > n
    for n, T, P in [(11, 2, 3), (20, 3, 4), (33, 1, 5)]:
        for c in range(0, n + 2):
            owner, count = oracle.iteration_map(n, T, P, 0, c)
            assert np.all(count == 1)
            assert owner.tolist() == [_closed_form_owner(i, n, T, P, 0, c) for i in range(n)]


def test_thread_chunks_partition_and_order():
    for n, T, P, dc, c in TINY[::7]:
        owner, _ = oracle.iteration_map(n, T, P, dc, c)
        seen = np.zeros(n, dtype=int)
        for k in range(T):
            for t in range(P):
                ch = oracle.thread_chunks(n, T, P, dc, c, k, t)
                prev_hi = -1
                for lo, hi in ch:
                    assert lo < hi
                    assert lo >= prev_hi          # executed in increasing order
                    prev_hi = hi
                    if c > 0:
                        assert hi - lo <= c
                    assert np.all(owner[lo:hi] == k * P + t)
                    seen[lo:hi] += 1
        assert np.all(seen == 1)


def test_balanced_sizes_differ_by_at_most_one():
    for m, p in itertools.product(range(0, 40), range(1, 12)):
        sizes = [oracle.bal(m, p, t)[1] - oracle.bal(m, p, t)[0] for t in range(p)]
        assert sum(sizes) == m
        assert max(sizes) - min(sizes) <= 1
        assert sizes == sorted(sizes, reverse=True)     # larger shares first
        los = [oracle.bal(m, p, t)[0] for t in range(p)]
        assert los[0] == 0 and all(los[t + 1] == oracle.bal(m, p, t)[1] for t in range(p - 1))


def test_chunked_sizes_are_c_except_last_in_each_distribute_chunk():
    n, T, P, dc, c = 1000, 3, 4, 37, 5
    for k in range(T):
        for t in range(P):
            for lo, hi in oracle.thread_chunks(n, T, P, dc, c, k, t):
                blk_end = min(n, (lo // dc + 1) * dc)
                assert hi - lo == c or hi == blk_end


def test_round_robin_restarts_at_thread_zero_per_distribute_chunk():
    # every distribute chunk's first iteration is executed by thread 0
    n, T, P, dc, c = 500, 4, 3, 17, 2
    owner, _ = oracle.iteration_map(n, T, P, dc, c)
    for j in range(0, (n + dc - 1) // dc):
        assert owner[j * dc] % P == 0
        assert owner[j * dc] // P == j % T


def test_surplus_teams_and_threads_idle():
    owner, count = oracle.iteration_map(3, 8, 4, 0, 0)
    assert owner.tolist() == [0 * 4, 1 * 4, 2 * 4] and np.all(count == 1)
    assert oracle.thread_chunks(3, 8, 4, 0, 0, 5, 0) == []
    assert oracle.thread_chunks(3, 8, 4, 0, 0, 0, 1) == []


def test_deterministic():
    a = oracle.iteration_map(777, 5, 7, 3, 4)
    b = oracle.iteration_map(777, 5, 7, 3, 4)
    assert np.array_equal(a[0], b[0])


def test_bad_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.iteration_map(10, 0, 4)
    with pytest.raises(ValueError):
        oracle.iteration_map(10, 1, 4, 0, -1)


def test_hand_worked_2pow20_one_team_256_threads():
    g = json.load(open(GOLDEN))
    n, T, P = g["n"], g["teams"], g["threads"]
    # default chunk
    owner, count = oracle.iteration_map(n, T, P, 0, 0)
    assert np.all(count == 1)
    d = g["default_chunk"]
    for t, lo, hi in d["thread_ranges_sample"]:
        assert oracle.thread_chunks(n, T, P, 0, 0, 0, t) == [(lo, hi)]
    assert np.all(np.bincount(owner, minlength=P) == d["iters_per_thread"])
    assert owner[n - 1] == d["is_last_thread"]
    # chunk 7
    c7 = g["chunk_7"]
    owner, count = oracle.iteration_map(n, T, P, 0, 7)
    assert np.all(count == 1)
    nch = [len(oracle.thread_chunks(n, T, P, 0, 7, 0, t)) for t in range(P)]
    assert sum(nch) == c7["total_chunks"]
    assert all(v == c7["chunks_thread_0_to_36"] for v in nch[:37])
    assert all(v == c7["chunks_thread_37_to_255"] for v in nch[37:])
    last = oracle.thread_chunks(n, T, P, 0, 7, 0, c7["last_chunk_thread"])[-1]
    assert list(last) == c7["last_chunk"]
    assert owner[n - 1] == c7["last_chunk_thread"]
    it = np.bincount(owner, minlength=P)
    assert it[0] == c7["iters_thread_0"] and it[36] == c7["iters_thread_36"]
    assert it[37] == c7["iters_thread_37"]
    assert oracle.thread_chunks(n, T, P, 0, 7, 0, 1)[:2] == [tuple(x) for x in c7["first_chunks_thread_1"]]
