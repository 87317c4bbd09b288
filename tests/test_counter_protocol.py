"""Host model of the cross-team combine protocol (CPU only).

Every team publishes its partial, then performs the wrap-around atomic
increment the paper describes for ``inc`` (sec. 3.1/3.2): it returns the old
value v and stores ``0 if v >= e else v + 1``.  With e = T - 1 the team that
reads T - 1 is the last to arrive, and it leaves the counter at 0, so the
next launch (or graph replay) needs no reset.  This model runs every arrival
order for small T, repeated launches, and the batched form where segment s
has its own counter with e = tiles_s - 1.
"""
import itertools

import numpy as np


def atomic_inc(mem, addr, e):
    v = mem[addr]
    mem[addr] = 0 if v >= e else v + 1
    return v


def run_launch(order, partials, mem, addr=0):
    T = len(partials)
    published = {}
    last = []
    for k in order:
        published[k] = partials[k]            # store, then release fence
        if atomic_inc(mem, addr, T - 1) == T - 1:
            # acquire: every team's store precedes its increment, all T seen
            assert len(published) == T
            last.append(sum(published[j] for j in range(T)))
    return last


def test_all_arrival_orders_small_T():
    for T in range(1, 6):
        partials = list(range(10, 10 + T))
        for order in itertools.permutations(range(T)):
            mem = [0]
            last = run_launch(order, partials, mem)
            assert last == [sum(partials)]     # exactly one last team, full sum
            assert mem[0] == 0                 # counter reset by the wrap


def test_repeated_launches_self_reset():
    g = np.random.Generator(np.random.PCG64(0))
    mem = [0]
    for rep in range(200):
        T = int(g.integers(1, 9))
        order = g.permutation(T)
        partials = g.integers(-100, 100, T).tolist()
        assert run_launch(order, partials, mem) == [sum(partials)]
        assert mem[0] == 0


def test_batched_per_segment_counters_interleaved():
    g = np.random.Generator(np.random.PCG64(1))
    tiles = [1, 3, 5, 2, 7]
    mem = [0] * len(tiles)
    for rep in range(20):
        events = [(s, t) for s, n in enumerate(tiles) for t in range(n)]
        g.shuffle(events)
        lasts = []
        for s, t in events:
            if atomic_inc(mem, s, tiles[s] - 1) == tiles[s] - 1:
                lasts.append(s)
        assert sorted(lasts) == list(range(len(tiles)))
        assert mem == [0] * len(tiles)


def test_nonzero_counter_is_detectable():
    # a counter left non-zero (aborted launch) makes the wrong team "last";
    # the library's reset entry point exists for that case
    mem = [2]
    order = [0, 1, 2, 3]
    seen = []
    for k in order:
        if atomic_inc(mem, 0, 3) == 3:
            seen.append(k)
    assert seen == [1] and mem[0] == 2
