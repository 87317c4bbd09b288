"""Pins for the oracle's dynamic / guided worksharing queues (CPU only).

The chunk sequences below are worked out by hand from the rules: dynamic
hands out chunks of c iterations in order; guided hands out ceil(r / P) of
the r remaining iterations, at least c and at most r.  Invariants and
special cases (P = 1, c >= m, empty blocks, per-block queues under
dist_schedule) cover the rest.
"""
import numpy as np
import pytest

import oracle


def sizes(ch):
    return [h - l for l, h in ch]


def test_guided_worked_example_c1():
    ch = oracle.queue_chunks("guided", 100, 4, 1)
    assert sizes(ch) == [25, 19, 14, 11, 8, 6, 5, 3, 3, 2, 1, 1, 1, 1]
    assert ch[0] == (0, 25) and ch[3] == (58, 69) and ch[-1] == (99, 100)


def test_guided_worked_example_c4_and_small():
    assert sizes(oracle.queue_chunks("guided", 100, 4, 4)) == [25, 19, 14, 11, 8, 6, 5, 4, 4, 4]
    assert sizes(oracle.queue_chunks("guided", 10, 4, 0)) == [3, 2, 2, 1, 1, 1]
    # the last chunk may be shorter than c
    assert sizes(oracle.queue_chunks("guided", 10, 4, 3)) == [3, 3, 3, 1]


def test_dynamic_chunks():
    assert oracle.queue_chunks("dynamic", 10, 4, 3) == [(0, 3), (3, 6), (6, 9), (9, 10)]
    assert oracle.queue_chunks("dynamic", 5, 64, 0) == [(i, i + 1) for i in range(5)]
    assert len(oracle.queue_chunks("dynamic", 1 << 20, 256, 64)) == (1 << 20) // 64


def test_special_cases():
    assert oracle.queue_chunks("guided", 1000, 1, 1) == [(0, 1000)]     # one thread: one chunk
    assert oracle.queue_chunks("guided", 7, 4, 10) == [(0, 7)]         # c >= m
    assert oracle.queue_chunks("dynamic", 0, 4, 1) == []
    assert oracle.queue_chunks("guided", 0, 4, 1) == []


@pytest.mark.parametrize("m,P,c", [(1, 1, 0), (1000, 7, 0), (12345, 256, 1), (12345, 256, 64),
                                   (1 << 20, 1024, 0), (999, 1000, 5)])
def test_guided_invariants(m, P, c):
    ch = oracle.queue_chunks("guided", m, P, c)
    s = sizes(ch)
    cmin = max(c, 1)
    assert ch[0][0] == 0 and ch[-1][1] == m
    assert all(ch[i][1] == ch[i + 1][0] for i in range(len(ch) - 1))   # contiguous, in order
    assert s[0] == min(m, max(cmin, -(-m // P)))
    assert all(a >= b for a, b in zip(s, s[1:]))                       # non-increasing
    assert all(x >= cmin for x in s[:-1])
    # each chunk is the share of what was left when it was taken
    left = m
    for x in s:
        assert x == min(left, max(cmin, -(-left // P)))
        left -= x


def test_team_queue_restarts_per_block():
    # dist_schedule(static, 10) over 35 iterations, 2 teams: team 0 has blocks [0,10), [20,30)
    q = oracle.team_queue("dynamic", 35, 2, 4, 10, 4, 0)
    assert q == [(0, 4), (4, 8), (8, 10), (20, 24), (24, 28), (28, 30)]
    q = oracle.team_queue("guided", 35, 2, 4, 10, 1, 1)       # blocks [10,20), [30,35)
    assert q == [(10, 13), (13, 15), (15, 17), (17, 18), (18, 19), (19, 20), (30, 32), (32, 33),
                 (33, 34), (34, 35)]
    # balanced blocks: 3 teams over 10 -> [0,4), [4,7), [7,10); surplus teams have no queue
    assert oracle.team_queue("dynamic", 10, 3, 2, 0, 0, 1) == [(4, 5), (5, 6), (6, 7)]
    assert oracle.team_queue("guided", 2, 4, 8, 0, 0, 3) == []


def test_every_iteration_in_exactly_one_chunk():
    n, T, P = 100003, 13, 96
    for kind in ("dynamic", "guided"):
        for dc, c in ((0, 0), (0, 7), (1000, 3), (777, 0)):
            hit = np.zeros(n, dtype=np.int64)
            for k in range(T):
                for l, h in oracle.team_queue(kind, n, T, P, dc, c, k):
                    hit[l:h] += 1
            assert np.all(hit == 1), (kind, dc, c)
