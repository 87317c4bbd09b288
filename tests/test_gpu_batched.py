"""GPU parity of the batched persistent launch (graph captured once, then
replayed) against the oracle per segment, plus the plain one-launch-per-
segment form; both ticket and round-robin tile dealing; replays without
any counter reset.
"""
from concurrent.futures import ThreadPoolExecutor

import pytest
import torch

import synth
from gpu_util import check_value, identity, oracle_value, to_device, to_host, x_tensor, x_value

pytestmark = pytest.mark.gpu

OPN = {synth.SUM: "sum", synth.MAX: "max", synth.MIN: "min"}


def _make(count, seed, lo_exp, hi_exp, dtypes=(synth.I64, synth.F32, synth.BF16)):
    lens, dts, ops = synth.batched_spec(count, seed, lo_exp, hi_exp, dtypes)
    ins, xs, meta = [], [], []
    for i in range(count):
        n, dt, op = int(lens[i]), int(dts[i]), OPN[int(ops[i])]
        host = synth.host(dt, n, 10_000 + i)
        ins.append(to_device(host, dt))
        x0 = identity(dt, op) if i % 2 == 0 else (3 if dt in (synth.I32, synth.I64) else 0.5)
        xs.append(x_tensor(dt, op, x0))
        meta.append((host, dt, op, x0))
    return ins, xs, meta


def _check_all(xs, meta):
    torch.cuda.synchronize()
    for x, (host, dt, op, x0) in zip(xs, meta):
        ref, sabs = oracle_value(host, dt, op, x0)
        check_value(x_value(x), ref, sabs, dt, op)


def _reset(xs, meta):
    for x, (_, dt, op, x0) in zip(xs, meta):
        x.copy_(x_tensor(dt, op, x0))


@pytest.mark.parametrize("config", [None, {"tile_kib": 16}, {"tile_kib": 64, "threads": 512, "unroll": 8},
                                    {"tile_kib": 32, "flags": 2, "teams": 37},
                                    {"tile_kib": 8, "vec": 8, "unroll": 2, "threads": 128}])
def test_batched_mixed_segments_replayed(gpu_lib, config):
    om = gpu_lib
    ins, xs, meta = _make(300, 61, 0.0, 5.3, (synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16))
    segs = om.make_segments([(i, m[2], x) for i, x, m in zip(ins, xs, meta)])
    for rep in range(3):
        _reset(xs, meta)
        om.reduce_batched(segs, config=config)
        _check_all(xs, meta)


def test_reduce_each_matches_oracle(gpu_lib):
    om = gpu_lib
    ins, xs, meta = _make(200, 62, 2.0, 5.0)
    segs = om.make_segments([(i, m[2], x) for i, x, m in zip(ins, xs, meta)])
    om.reduce_each(segs)
    _check_all(xs, meta)


def test_batched_empty_and_single(gpu_lib):
    om = gpu_lib
    a = torch.arange(10, dtype=torch.int64, device="cuda")
    x = torch.zeros(1, dtype=torch.int64, device="cuda")
    y = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    om.reduce_batched([(a, "sum", x), (a[:0], "sum", y, 0)])
    torch.cuda.synchronize()
    assert x.item() == 45 and y.item() == 5


def test_batched_many_replays_no_reset(gpu_lib):
    om = gpu_lib
    ins, xs, meta = _make(64, 63, 3.0, 6.0, (synth.I64,))
    segs = om.make_segments([(i, "sum", x) for i, x in zip(ins, xs)])
    for x in xs:
        x.zero_()
    reps = 200
    for _ in range(reps):
        om.reduce_batched(segs, config={"tile_kib": 16})
    torch.cuda.synchronize()
    for x, (host, _, _, _) in zip(xs, meta):
        s = int(host.astype(object).sum())
        want = (reps * s + 2**63) % 2**64 - 2**63
        assert x.item() == want
    assert om.workspace_status() == 0


def check_every_segment(ins, xs, info, x0s=None, what=""):
    """Every segment's result against the oracle, from host copies, several segments at
    a time (the oracle's C loops run outside the interpreter lock).  Returns the
    (rel, kappa) records of the floating sums."""
    torch.cuda.synchronize()

    def one(i):
        dt, op = info[i]
        x0 = identity(dt, op) if x0s is None else x0s[i]
        ref, sabs = oracle_value(to_host(ins[i]), dt, op, x0)
        return check_value(x_value(xs[i]), ref, sabs, dt, op, f"{what} segment {i}",
                           n=int(ins[i].numel()))

    with ThreadPoolExecutor(8) as ex:
        return [r for r in ex.map(one, range(len(ins))) if r is not None]


@pytest.mark.slow
def test_batched_full_4096_every_segment(gpu_lib):
    """4096 segments, lengths log-uniform in [1e2, 1e7] (about 16 GB), int64 / fp32 /
    bf16, sum / max / min: every segment of the persistent graph-replayed launch, and
    of the plain one-launch-per-segment form, against the oracle."""
    om = gpu_lib
    lens, dts, ops = synth.batched_spec(4096, synth.SEED_BATCH)
    ins, xs, info = [], [], []
    for i in range(4096):
        dt, op = int(dts[i]), OPN[int(ops[i])]
        ins.append(synth.device(dt, int(lens[i]), 20_000 + i))
        xs.append(x_tensor(dt, op, identity(dt, op)))
        info.append((dt, op))
    segs = om.make_segments([(t, op, x) for t, x, (dt, op) in zip(ins, xs, info)])
    om.reduce_batched(segs)
    om.reduce_batched(segs)           # a replay of the cached graph, from the identity again
    for x, (dt, op) in zip(xs, info):
        x.copy_(x_tensor(dt, op, identity(dt, op)))
    om.reduce_batched(segs)
    errs = check_every_segment(ins, xs, info, what="batched")
    assert len(errs) == sum(1 for dt, op in info if op == "sum" and dt != synth.I64)
    for x, (dt, op) in zip(xs, info):
        x.copy_(x_tensor(dt, op, identity(dt, op)))
    om.reduce_each(segs)
    check_every_segment(ins, xs, info, what="plain")
    assert om.workspace_status() == 0
