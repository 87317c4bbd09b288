"""Host checks of dynamic / guided worksharing (no GPU).

* omprt_queue_chunk (host arithmetic of the library) against the oracle's
  chunk sequences;
* a CPU model of the kernel's wave-at-a-time queue: random orders of wave
  requests, each taking tickets for all of the wave's active lanes with one
  add.  Whatever the order, every chunk number must go to exactly one lane;
* argument errors of the new entry points.
"""
import ctypes
import random

import pytest

import oracle
import paper_2106_03219_amd as om
from paper_2106_03219_amd import _lib


@pytest.mark.parametrize("kind", ["dynamic", "guided"])
@pytest.mark.parametrize("m,P,c", [(0, 4, 1), (1, 1, 0), (100, 4, 1), (100, 4, 4), (12345, 256, 0),
                                   (12345, 96, 7), (1 << 20, 512, 0), (999, 1000, 5)])
def test_library_queue_chunks_match_oracle(kind, m, P, c):
    want = oracle.queue_chunks(kind, m, P, c)
    got = []
    j = 0
    while True:
        lo, hi = om.queue_chunk(kind, m, P, c, j)
        if lo == hi:
            assert lo == m
            break
        got.append((lo, hi))
        j += 1
    assert got == want


def model_queue(kind, m, P, c, waves, tickets, rng):
    """Chunk numbers each (wave, lane) receives under one random order of wave requests:
    the wave's active lanes take cnt * tickets numbers with one add, lane r getting
    base + r + j * cnt; a lane whose first number is past the end leaves."""
    nch = len(oracle.queue_chunks(kind, m, P, c))
    q = 0
    active = {w: list(range(min(64, P - 64 * w))) for w in range(waves)}
    got = []
    while active:
        w = rng.choice(sorted(active))
        lanes = active[w]
        base = q
        q += len(lanes) * tickets
        keep = []
        for rank, lane in enumerate(lanes):
            first = base + rank
            if first >= nch:
                continue
            keep.append(lane)
            for j in range(tickets):
                t = first + j * len(lanes)
                if t < nch:
                    got.append(((w, lane), t))
        if keep:
            active[w] = keep
        else:
            del active[w]
    return got, nch


@pytest.mark.parametrize("kind", ["dynamic", "guided"])
@pytest.mark.parametrize("tickets", [1, 4])
@pytest.mark.parametrize("m,P,c", [(1, 64, 0), (100, 4, 1), (5000, 96, 0), (5000, 256, 3),
                                   (20000, 512, 64), (777, 130, 0)])
def test_wave_model_hands_out_every_chunk_once(kind, tickets, m, P, c):
    rng = random.Random(m * 31 + P)
    waves = -(-P // 64)
    for _ in range(5):
        got, nch = model_queue(kind, m, P, c, waves, tickets, rng)
        assert sorted(t for _, t in got) == list(range(nch))


def test_argument_errors():
    lib = _lib.load()
    lb, ub = ctypes.c_int64(), ctypes.c_int64()
    assert lib.omprt_queue_chunk(3, 10, 4, 1, 0, ctypes.byref(lb), ctypes.byref(ub)) == _lib.ERR_INVALID
    assert lib.omprt_queue_chunk(1, -1, 4, 1, 0, ctypes.byref(lb), ctypes.byref(ub)) == _lib.ERR_INVALID
    assert lib.omprt_queue_chunk(1, 10, 0, 1, 0, ctypes.byref(lb), ctypes.byref(ub)) == _lib.ERR_INVALID
    assert lib.omprt_queue_chunk(1, 10, 4, 1, -1, ctypes.byref(lb), ctypes.byref(ub)) == _lib.ERR_INVALID
    assert lib.omprt_queue_chunk(2, 10, 4, 1, 0, None, ctypes.byref(ub)) == _lib.ERR_INVALID
    s = _lib.Sched(100, 2, 64, 0, 1)
    assert lib.omprt_queue_map(ctypes.byref(s), 0, 1, None, None, None, None) == _lib.ERR_INVALID
    assert lib.omprt_queue_map(ctypes.byref(s), 2, 65, None, None, None, None) == _lib.ERR_INVALID
    assert lib.omprt_queue_map(ctypes.byref(s), 1, 0, None, None, None, None) == _lib.ERR_INVALID
    assert lib.omprt_queue_map(ctypes.byref(s), 1, 1, None, None, None, None) == _lib.ERR_INVALID
    s0 = _lib.Sched(0, 2, 64, 0, 1)
    assert lib.omprt_queue_map(ctypes.byref(s0), 1, 1, None, None, None, None) == _lib.OK
    assert lib.omprt_axpy_sum_queue(ctypes.c_float(1.0), None, None, None, ctypes.byref(s), 1, None) == _lib.ERR_INVALID
    x = ctypes.c_float(0)
    assert lib.omprt_axpy_sum_queue(ctypes.c_float(1.0), None, None, ctypes.byref(x), ctypes.byref(s), 5, None) == _lib.ERR_INVALID
    assert lib.omprt_axpy_sum_queue(ctypes.c_float(1.0), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1100),
                                    ctypes.byref(x), ctypes.byref(s), 1, None) == _lib.ERR_INVALID   # overlap
