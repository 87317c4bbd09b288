"""GPU parity of the plain paths against the oracle, through the C ABI.

Covers: the int32 2^20 reduction and the 1 x 256 static map (default chunk
and chunk 7) bit-exact; every dtype x op on ragged, misaligned sizes over
several configurations; the 2^28 fp32 sum / max and int64 sum over the
team sweep 1..2048 x 256 in the benchmark's launch configuration; x_orig
handling, n = 0, determinism; iteration maps of many schedules; the
cross-team protocol under 10^4 back-to-back launches.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (OPS, check_value, identity, oracle_value, to_device, to_host, x_tensor,
                      x_value)

pytestmark = pytest.mark.gpu


def _reduce_and_check(om, host, dtype, op, x0, config=None, offset=0, what=""):
    dev = to_device(host, dtype)
    inp = dev[offset:]
    x = x_tensor(dtype, op, x0)
    om.reduce(inp, op, x, config=config)
    torch.cuda.synchronize()
    ref, sabs = oracle_value(host[offset:], dtype, op, x0)
    check_value(x_value(x), ref, sabs, dtype, op, what)
    return x_value(x)


# ---------------------------------------------------------------- C1

def test_int32_2pow20_sum_one_team_and_auto(gpu_lib):
    om = gpu_lib
    host = synth.int32_uniform(1 << 20, synth.SEED_C1)
    ref = oracle.reduce_int(host, "sum", 0)
    dev = to_device(host, synth.I32)
    for cfg in ({"teams": 1, "threads": 256}, None, {"teams": 256, "threads": 256}):
        x = torch.zeros(1, dtype=torch.int32, device="cuda")
        om.reduce(dev, "sum", x, config=cfg)
        torch.cuda.synchronize()
        assert int(x.item()) == ref, cfg


@pytest.mark.parametrize("chunk", [0, 7])
def test_static_map_2pow20_one_team_256(gpu_lib, chunk):
    om = gpu_lib
    n = 1 << 20
    owner = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    count = torch.zeros(n, dtype=torch.int32, device="cuda")
    om.static_map(n, 1, 256, 0, chunk, owner, count)
    torch.cuda.synchronize()
    ro, rc = oracle.iteration_map(n, 1, 256, 0, chunk)
    assert np.array_equal(owner.cpu().numpy(), ro)
    assert np.array_equal(count.cpu().numpy().view(np.uint32), rc)


MAPS = [(0, 1, 1, 0, 0), (1, 1, 1, 0, 0), (100, 3, 64, 0, 0), (1000, 7, 9, 0, 0), (1000, 7, 9, 0, 3),
        (1000, 4, 100, 13, 0), (1000, 4, 100, 13, 5), (5, 8, 64, 0, 0), (12345, 5, 256, 1000, 64),
        (100000, 64, 256, 0, 1), (100000, 64, 256, 0, 1024), (100000, 33, 1024, 777, 7),
        (70000, 4096, 64, 0, 0)]


@pytest.mark.parametrize("n,T,P,dc,c", MAPS)
def test_static_map_schedules(gpu_lib, n, T, P, dc, c):
    om = gpu_lib
    owner = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    count = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    om.static_map(n, T, P, dc, c, owner, count)
    torch.cuda.synchronize()
    ro, rc = oracle.iteration_map(n, T, P, dc, c)
    assert np.array_equal(owner.cpu().numpy()[:n], ro)
    assert np.array_equal(count.cpu().numpy()[:n].view(np.uint32), rc)


# ---------------------------------------------------------------- all dtypes x ops, ragged

RAGGED_N = [1, 2, 3, 63, 64, 65, 1000, 4097, 65537, 1 << 20 | 12345]
CONFIGS = [None, {"teams": 1, "threads": 64, "vec": 16, "unroll": 1},
           {"teams": 3, "threads": 128, "vec": 8, "unroll": 2},
           {"teams": 300, "threads": 256, "vec": 16, "unroll": 8},
           {"teams": 64, "threads": 1024, "vec": 16, "unroll": 4}]


@pytest.mark.parametrize("dtype", [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16])
def test_all_dtypes_ops_ragged(gpu_lib, dtype):
    om = gpu_lib
    g = np.random.Generator(np.random.PCG64(100 + dtype))
    for n in RAGGED_N:
        host = synth.host(dtype, n + 3, 1000 + n)
        for op in OPS:
            cfg = CONFIGS[int(g.integers(0, len(CONFIGS)))]
            offset = int(g.integers(0, 4))          # misaligned starts
            _reduce_and_check(om, host, dtype, op, identity(dtype, op), cfg, offset,
                              f"dt={dtype} n={n} op={op} cfg={cfg} off={offset}")


@pytest.mark.parametrize("dtype", [synth.I32, synth.I64, synth.F32, synth.BF16])
def test_nonzero_x_orig_and_empty(gpu_lib, dtype):
    om = gpu_lib
    host = synth.host(dtype, 5000, 77)
    big = {synth.I32: 999999, synth.I64: 2**41}.get(dtype, 1e3)   # beyond the data's range
    xs = {"sum": 5 if dtype in (synth.I32, synth.I64) else 2.5, "max": big, "min": -big}
    for op in OPS:
        got = _reduce_and_check(om, host, dtype, op, xs[op], None, 0, f"x_orig {op}")
        if op != "sum":
            assert got == xs[op]
        x = x_tensor(dtype, op, xs[op])
        om.reduce(to_device(host, dtype), op, x, n=0)
        torch.cuda.synchronize()
        assert x_value(x) == xs[op]


def test_planted_extremes_and_int_wrap(gpu_lib):
    om = gpu_lib
    a = synth.f32_normal(1 << 22, 9)
    a[3_000_001] = 77.5
    a[17] = -88.25
    _reduce_and_check(om, a, synth.F32, "max", -np.inf)
    _reduce_and_check(om, a, synth.F32, "min", np.inf)
    w = np.full(1 << 20, 1 << 12, dtype=np.int32)            # sums to 2^32 == 0
    w[5] += 3
    _reduce_and_check(om, w, synth.I32, "sum", 0)
    big = np.full(1 << 16, 2**62, dtype=np.int64)
    _reduce_and_check(om, big, synth.I64, "sum", 7)
    ones = np.ones((1 << 24) + 1000, dtype=np.float32)        # exact only with compensation / tree
    _reduce_and_check(om, ones, synth.F32, "sum", 0.0)
    spike = np.concatenate([np.array([1e8], dtype=np.float32), np.ones(1 << 20, dtype=np.float32)])
    _reduce_and_check(om, spike, synth.F32, "sum", 0.0, {"teams": 1, "threads": 64, "vec": 16, "unroll": 1})


def test_deterministic_for_fixed_config(gpu_lib):
    om = gpu_lib
    host = synth.f32_normal(3_000_017, 5)
    dev = to_device(host, synth.F32)
    outs = set()
    for _ in range(5):
        x = torch.zeros(1, dtype=torch.float32, device="cuda")
        om.reduce(dev, "sum", x, config={"teams": 512, "threads": 256, "vec": 16, "unroll": 4})
        torch.cuda.synchronize()
        outs.add(x.view(torch.int32).item())
    assert len(outs) == 1


# ---------------------------------------------------------------- 2^28 at scale

@pytest.fixture(scope="module")
def big_inputs():
    n = 1 << 28
    f = synth.device(synth.F32, n, synth.SEED_F32)
    i = synth.device(synth.I64, n, synth.SEED_I64)
    fh, ih = to_host(f), to_host(i)
    refs = {
        ("f32", "sum"): oracle.reduce_fp(fh, "sum", 0.0, want_abs=True),
        ("f32", "max"): (oracle.reduce_fp(fh, "max", -np.inf), None),
        ("i64", "sum"): (oracle.reduce_int(ih, "sum", 0), None),
    }
    del fh, ih
    yield f, i, refs
    del f, i
    torch.cuda.empty_cache()


@pytest.mark.parametrize("teams", [1, 8, 64, 256, 512, 1024, 2048])
def test_2pow28_team_sweep(gpu_lib, big_inputs, teams):
    om = gpu_lib
    f, i, refs = big_inputs
    cfg = {"teams": teams, "threads": 256}
    for key, t, dt, op in [(("f32", "sum"), f, synth.F32, "sum"), (("f32", "max"), f, synth.F32, "max"),
                           (("i64", "sum"), i, synth.I64, "sum")]:
        x = x_tensor(dt, op, identity(dt, op))
        om.reduce(t, op, x, config=cfg)
        torch.cuda.synchronize()
        ref, sabs = refs[key]
        check_value(x_value(x), ref, sabs, dt, op, f"{key} T={teams}")


def test_2pow28_default_config(gpu_lib, big_inputs):
    om = gpu_lib
    f, i, refs = big_inputs
    x = torch.zeros(1, dtype=torch.float32, device="cuda")
    om.reduce(f, "sum", x)
    y = torch.zeros(1, dtype=torch.int64, device="cuda")
    om.reduce(i, "sum", y)
    torch.cuda.synchronize()
    check_value(x.item(), refs[("f32", "sum")][0], refs[("f32", "sum")][1], synth.F32, "sum")
    assert y.item() == refs[("i64", "sum")][0]


# ---------------------------------------------------------------- protocol stress

def test_back_to_back_launches_self_reset(gpu_lib):
    om = gpu_lib
    ones = torch.ones(5000, dtype=torch.int64, device="cuda")
    x = torch.zeros(1, dtype=torch.int64, device="cuda")
    reps = 10000
    for _ in range(reps):
        om.reduce(ones, "sum", x, config={"teams": 4096, "threads": 64, "vec": 16, "unroll": 1})
    torch.cuda.synchronize()
    assert x.item() == reps * 5000
    # alternating team counts on the same stream share the counter safely
    y = torch.zeros(1, dtype=torch.int64, device="cuda")
    for r in range(1000):
        om.reduce(ones, "sum", y, config={"teams": 1 + (r * 37) % 2048, "threads": 64})
    torch.cuda.synchronize()
    assert y.item() == 1000 * 5000
    assert om.workspace_status() == 0      # no last team ever gave up waiting


def test_separate_streams(gpu_lib):
    om = gpu_lib
    a = torch.arange(100000, dtype=torch.int64, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    x1 = torch.zeros(1, dtype=torch.int64, device="cuda")
    x2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    for _ in range(200):
        om.reduce(a, "sum", x1, config={"teams": 700, "threads": 128}, stream=s1)
        om.reduce(a, "sum", x2, config={"teams": 900, "threads": 256}, stream=s2)
    torch.cuda.synchronize()
    assert x1.item() == x2.item() == 200 * (100000 * 99999 // 2)


def test_empty_region_sweep(gpu_lib):
    """Empty regions over N in {0, 1, 2, 4, ..., 1024} (plus two large trip counts) for
    T in 1..64 teams and several (P, dist_chunk, chunk) schedules: every launch must
    count exactly N iterations through its team tree and cross-team step, and no
    thread may find its chunks inconsistent (status bit 16)."""
    om = gpu_lib
    om.workspace_reset()
    assert om.workspace_status() == 0
    ns = [0] + [1 << k for k in range(11)] + [3, 1000, 1023, (1 << 40) + 12345]
    teams = (1, 2, 3, 8, 17, 64)
    scheds = [(256, 0, 0), (256, 0, 1), (256, 0, 7), (100, 3, 2), (64, 5, 0), (1, 1, 1),
              (1024, 1024, 64), (33, 0, 1024)]
    cases = [(n, T, P, dc, c) for n in ns for T in teams for (P, dc, c) in scheds
             if not (n > 1 << 20 and dc and dc < 1024)]
    iters = torch.zeros(len(cases), dtype=torch.int64, device="cuda")
    for k, (n, T, P, dc, c) in enumerate(cases):
        om.empty_region(n, T, P, dc, c, iters=iters[k:k + 1])
    assert om.workspace_status() == 0
    got = iters.cpu().tolist()
    bad = [(case, g) for case, g in zip(cases, got) if g != case[0]]
    assert not bad, bad[:10]
    # without a counter the region still runs the whole protocol
    for T in (1, 64):
        om.empty_region(1024, T, 256)
    assert om.workspace_status() == 0


def test_plain_launches_under_caller_graph_capture(gpu_lib):
    """Multi-team reductions captured into a caller's HIP graph and replayed many times,
    with eager work between replays: every replay must reproduce the eager result
    (the cross-team tags come from device memory, so replays never see stale slots)."""
    om = gpu_lib
    f = to_device(synth.f32_normal(3_000_001, 31), synth.F32)
    i = to_device(synth.int64_uniform(2_000_003, 32), synth.I64)
    s = torch.cuda.Stream()
    om.workspace_reserve(4096, stream=s)
    xs = torch.zeros(1, dtype=torch.float32, device="cuda")
    xi = torch.zeros(1, dtype=torch.int64, device="cuda")
    xm = torch.full((1,), -float("inf"), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    # eager reference on the same stream and configurations
    with torch.cuda.stream(s):
        om.reduce(f, "sum", xs, config={"teams": 777, "threads": 256})
        om.reduce(i, "sum", xi, config={"teams": 1500, "threads": 512})
        om.reduce(f, "max", xm, config={"teams": 300, "threads": 1024})
    torch.cuda.synchronize()
    want = (xs.item(), xi.item(), xm.item())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        om.reduce(f, "sum", xs, config={"teams": 777, "threads": 256})
        om.reduce(i, "sum", xi, config={"teams": 1500, "threads": 512})
        om.reduce(f, "max", xm, config={"teams": 300, "threads": 1024})
    for rep in range(50):
        xs.zero_(); xi.zero_(); xm.fill_(-float("inf"))
        # unrelated eager launches on the default stream in between
        om.reduce(f, "sum", torch.zeros(1, dtype=torch.float32, device="cuda"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (xs.item(), xi.item(), xm.item()) == want, rep
    assert om.workspace_status(stream=s) == 0


def test_captured_graph_survives_workspace_growth(gpu_lib):
    """A graph captured at 777 teams, then an eager 8000-team call on the same stream
    (which outgrows the stream's workspace): the replays after the growth still run on
    the workspace they captured, which the library keeps until omprt_finalize, and
    reproduce the eager result."""
    om = gpu_lib
    f = to_device(synth.f32_normal(2_000_003, 34), synth.F32)
    s = torch.cuda.Stream()
    om.workspace_reserve(777, stream=s)
    xs = torch.zeros(1, dtype=torch.float32, device="cuda")
    cfg = {"teams": 777, "threads": 256}
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        om.reduce(f, "sum", xs, config=cfg)
    torch.cuda.synchronize()
    want = xs.item()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        om.reduce(f, "sum", xs, config=cfg)
    xs.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    assert xs.item() == want
    x2 = torch.zeros(1, dtype=torch.float32, device="cuda")
    with torch.cuda.stream(s):
        om.reduce(f, "sum", x2, config={"teams": 8000, "threads": 256})
    torch.cuda.synchronize()
    ref, sabs = oracle_value(to_host(f), synth.F32, "sum", 0.0)
    check_value(x2.item(), ref, sabs, synth.F32, "sum", "8000 teams")
    for rep in range(5):
        xs.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert xs.item() == want, rep
        with torch.cuda.stream(s):       # eager work on the grown workspace in between
            om.reduce(f, "sum", x2, config={"teams": 8000, "threads": 256})
    assert om.workspace_status(stream=s) == 0


@pytest.mark.slow
def test_max_sizes(gpu_lib):
    """Past 2^31 elements (64-bit indexing end to end) and the largest team count."""
    om = gpu_lib
    n = (1 << 31) + 12345
    b = synth.device(synth.BF16, n, 77)
    x = torch.zeros(1, dtype=torch.float32, device="cuda")
    om.reduce(b, "sum", x)
    xm = torch.full((1,), -float("inf"), dtype=torch.bfloat16, device="cuda")
    om.reduce(b, "max", xm)
    torch.cuda.synchronize()
    h = to_host(b)
    ref, sabs = oracle.reduce_fp(h, "sum", 0.0, bf16=True, want_abs=True)
    check_value(x.item(), ref, sabs, synth.BF16, "sum", "bf16 sum 2^31+12345")
    assert float(xm.float().item()) == oracle.reduce_fp(h, "max", -np.inf, bf16=True)
    del b, h
    torch.cuda.empty_cache()
    a = synth.int64_uniform(1_000_003, 78)
    ref = oracle.reduce_int(a, "sum", 0)
    y = torch.zeros(1, dtype=torch.int64, device="cuda")
    om.reduce(to_device(a, synth.I64), "sum", y, config={"teams": 65535, "threads": 64})
    torch.cuda.synchronize()
    assert y.item() == ref


# ---------------------------------------------------------------- exact thread map

@pytest.mark.parametrize("dtype", [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16])
def test_exact_thread_map_matches_oracle(gpu_lib, dtype):
    """EXACT_THREAD_MAP (every thread reduces its schedule(static) run): every op on ragged
    and misaligned sizes under several team shapes, against the oracle; integers, max and min
    also equal to the interleaved kernel's bits."""
    om = gpu_lib
    flag = om.CFG_EXACT_THREAD_MAP
    for k, n in enumerate([1, 3, 64, 1000, 4099, 65537, (1 << 20) + 7]):
        host = synth.host(dtype, n + 1, 900 + k)
        for op in OPS:
            for cfg in ({"teams": 1, "threads": 64}, {"teams": 7, "threads": 256},
                        {"teams": 300, "threads": 1024}, {}):
                got = _reduce_and_check(om, host, dtype, op, identity(dtype, op),
                                        config=dict(cfg, flags=flag), offset=1,
                                        what=(n, op, cfg))
                if dtype in (synth.I32, synth.I64) or op != "sum":
                    plain = _reduce_and_check(om, host, dtype, op, identity(dtype, op),
                                              config=cfg or None, offset=1)
                    assert got == plain, (n, op, cfg, got, plain)
    with pytest.raises(om.OmprtError):
        x = torch.zeros(1, dtype=torch.int32, device="cuda")
        om.reduce(to_device(synth.host(synth.I32, 10, 1), synth.I32), "prod", x,
                  config={"flags": flag})


def test_exact_thread_map_2pow28(gpu_lib, big_inputs):
    om = gpu_lib
    f, i, refs = big_inputs
    for dev, dtype, key in ((f, synth.F32, "f32"), (i, synth.I64, "i64")):
        x = x_tensor(dtype, "sum", 0)
        om.reduce(dev, "sum", x, config={"flags": om.CFG_EXACT_THREAD_MAP})
        torch.cuda.synchronize()
        ref, sabs = refs[(key, "sum")]
        check_value(x_value(x), ref, sabs, dtype, "sum", "exact 2^28")
