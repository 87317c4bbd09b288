"""GPU parity of the device atomics (add, inc, max, exchange, cas).

Without contention (every operation on its own word) the result is unique
and compared with the oracle exactly.  With contention the hardware picks
the order; the checks are what any linearisation must satisfy: add returns
a prefix chain and ends at the total, inc with e = T-1 hands out 0..T-1 once
each and returns to 0 (the last-team election), max ends at the maximum,
exchange returns every written value but the last exactly once, and a
contended cas has exactly one winner.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def _host(t):
    return t.cpu().numpy().view(np.uint32)


def _run(om, op, target, index, e, d=None):
    tt, it, et = _dev(target), _dev(index), _dev(e)
    dt = _dev(d) if d is not None else None
    old = torch.zeros(len(index), dtype=torch.int32, device="cuda")
    om.atomic_apply(op, tt, it, et, old, d=dt)
    torch.cuda.synchronize()
    return _host(tt), _host(old)


@pytest.mark.parametrize("op", ["add", "inc", "max", "exchange", "cas"])
def test_uncontended_matches_oracle(gpu_lib, op):
    g = np.random.Generator(np.random.PCG64(11))
    n = 100_003
    target = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    index = g.permutation(n).astype(np.uint32)
    e = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    if op == "cas":       # half the operations expect the current value
        e[::2] = target[index[::2]]
    d = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    got_t, got_old = _run(gpu_lib, op, target, index, e, d)
    want_t, want_old, _ = oracle.atomic_serial(op, target, index, e, d)
    assert np.array_equal(got_t, want_t)
    assert np.array_equal(got_old, want_old)


def test_inc_election_under_contention(gpu_lib):
    T, groups = 97, 1000
    index = np.repeat(np.arange(groups), T).astype(np.uint32)
    np.random.Generator(np.random.PCG64(3)).shuffle(index)
    e = np.full(index.size, T - 1, np.uint32)
    t, old = _run(gpu_lib, "inc", np.zeros(groups, np.uint32), index, e)
    assert np.all(t == 0)
    for gi in range(groups):
        assert sorted(old[index == gi].tolist()) == list(range(T))


def test_add_is_a_linearised_chain(gpu_lib):
    g = np.random.Generator(np.random.PCG64(4))
    targets, n = 64, 200_000
    init = g.integers(0, 1000, targets).astype(np.uint32)
    index = g.integers(0, targets, n).astype(np.uint32)
    e = g.integers(1, 100, n).astype(np.uint32)
    t, old = _run(gpu_lib, "add", init, index, e)
    for k in range(targets):
        m = index == k
        o, ee = old[m].astype(np.int64), e[m].astype(np.int64)
        order = np.argsort(o)
        o, ee = o[order], ee[order]
        assert o[0] == init[k]
        assert np.array_equal(o[1:], o[:-1] + ee[:-1])      # each read = previous read + operand
        assert t[k] == (init[k] + ee.sum()) % 2**32


def test_max_exchange_cas_under_contention(gpu_lib):
    g = np.random.Generator(np.random.PCG64(5))
    targets, n = 16, 50_000
    index = g.integers(0, targets, n).astype(np.uint32)
    e = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    init = g.integers(0, 2**32, targets, dtype=np.uint64).astype(np.uint32)
    t, old = _run(gpu_lib, "max", init, index, e)
    for k in range(targets):
        m = index == k
        assert t[k] == max(int(init[k]), int(e[m].max()))
        assert np.all(old[m] <= t[k])
        assert set(old[m].tolist()) <= set(e[m].tolist()) | {int(init[k])}
    t, old = _run(gpu_lib, "exchange", init, index, e)
    for k in range(targets):
        m = index == k
        written = sorted(e[m].tolist() + [int(init[k])])
        seen = sorted(old[m].tolist() + [int(t[k])])
        assert written == seen
    # every operation tries init -> its own id; exactly one per target wins
    ids = np.arange(1, n + 1, dtype=np.uint32) + np.uint32(2**31)
    t, old = _run(gpu_lib, "cas", init, index, init[index], ids)
    for k in range(targets):
        m = np.where(index == k)[0]
        winners = m[old[m] == init[k]]
        assert len(winners) == 1
        assert t[k] == ids[winners[0]]
        assert np.all(old[m[m != winners[0]]] == ids[winners[0]])


def test_out_of_range_index_flagged(gpu_lib):
    om = gpu_lib
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        om.workspace_reset()
        tt = _dev([0, 0])
        old = torch.zeros(3, dtype=torch.int32, device="cuda")
        om.atomic_apply("add", tt, _dev([0, 5, 1]), _dev([1, 1, 1]), old)
    assert om.workspace_status(stream=s) & 2
    assert _host(old).tolist() == [0, 0xFFFFFFFF, 0] and _host(tt).tolist() == [1, 1]
    with torch.cuda.stream(s):
        om.workspace_reset()
    assert om.workspace_status(stream=s) == 0
