"""GPU parity of the array-section reduction reduction(op: x[0:m]) against
the oracle's column folds, through the C ABI.

Covers every dtype x op on ragged shapes (whole rows and column tiles, m from
1 to 20000, rows from 1 to 10^5), x_orig != identity, vector and element
loads (forced, and from a misaligned input), team counts from 1 to 4096 (one
and two levels of election groups), repeated launches (bit-identical, status
clean), and sampled columns of 2^28-element blocks in the default launch.
Tolerances are those of the scalar reduction (gpu_util).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import OPS, TORCH_DT, check_value, identity, to_device, to_host

pytestmark = pytest.mark.gpu

DTYPES = [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16]
ESIZE = {synth.I32: 4, synth.I64: 8, synth.F32: 4, synth.F64: 8, synth.BF16: 2}
SHAPES = [(1, 1), (5, 1), (3, 7), (1000, 3), (777, 8), (513, 100), (300, 256), (300, 257),
          (97, 1000), (50, 1001), (40, 4096), (9, 5000), (3, 20000), (2000, 33), (100000, 1),
          (4096, 64)]


def x_init(dtype, op, m, seed, plain=False):
    """Host x_orig: the identity (plain) or random values the fold can cross."""
    g = np.random.Generator(np.random.PCG64(seed))
    if plain:
        v = identity(dtype, op)
        if dtype in (synth.I32, synth.I64):
            return np.full(m, v, dtype=np.int32 if dtype == synth.I32 else np.int64)
        return np.full(m, v, dtype=np.float64)
    if dtype == synth.I32:
        return g.integers(-5000, 5000, m).astype(np.int32)
    if dtype == synth.I64:
        return g.integers(-(2**41), 2**41, m).astype(np.int64)
    v = g.standard_normal(m) * 2.0
    if dtype == synth.BF16 and op != "sum":   # x of a bf16 max/min is bf16
        return torch.tensor(v, dtype=torch.bfloat16).double().numpy()
    if dtype in (synth.F32, synth.BF16):      # float32 x (bf16 sums keep an fp32 x)
        return v.astype(np.float32).astype(np.float64)
    return v


def x_device(dtype, op, xh):
    if dtype == synth.BF16 and op == "sum":
        return torch.tensor(xh, dtype=torch.float32, device="cuda")
    if dtype in (synth.F32, synth.F64, synth.BF16):
        return torch.tensor(xh, dtype=TORCH_DT[dtype], device="cuda")
    return torch.from_numpy(xh.copy()).cuda()


def x_values(x):
    if x.dtype == torch.bfloat16:
        return x.float().cpu().numpy().astype(np.float64)
    return x.cpu().numpy()


def run_and_check(om, host2d, dtype, op, xh, config=None, inp=None, cols=None):
    rows, m = host2d.shape
    dev = to_device(host2d.reshape(-1), dtype) if inp is None else inp
    x = x_device(dtype, op, xh)
    om.reduce_array(dev, rows, m, op, x, config=config)
    torch.cuda.synchronize()
    got = x_values(x)
    cols = range(m) if cols is None else cols
    for j in cols:
        col = np.ascontiguousarray(host2d[:, j])
        x0 = xh[j]
        if dtype in (synth.I32, synth.I64):
            ref, sabs = oracle.reduce_int(col, op, int(x0)), None
        else:
            ref, sabs = oracle.reduce_fp(col, op, float(x0), bf16=dtype == synth.BF16, want_abs=True)
        check_value(got[j], ref, sabs, dtype, op, (rows, m, j, config))
    return got


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", OPS)
def test_ragged_shapes_default_launch(gpu_lib, dtype, op):
    for i, (rows, m) in enumerate(SHAPES):
        host = synth.host(dtype, rows * m, 1000 + i).reshape(rows, m)
        run_and_check(gpu_lib, host, dtype, op, x_init(dtype, op, m, 7 + i, plain=(i % 2 == 0)))


CONFIGS = [{"vec": 0}, {"teams": 1}, {"teams": 3}, {"teams": 4096}, {"threads": 64, "unroll": 1},
           {"threads": 512, "unroll": 1}, {"threads": 256, "teams": 512}, {"threads": 128, "unroll": 8}]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("cfg", range(len(CONFIGS) + 1))
def test_launch_configurations(gpu_lib, dtype, cfg):
    config = dict(CONFIGS[cfg]) if cfg < len(CONFIGS) else {"vec": ESIZE[dtype]}
    for i, (rows, m) in enumerate([(20000, 3), (2049, 64), (300, 257), (64, 4096), (5000, 1)]):
        host = synth.host(dtype, rows * m, 2000 + i).reshape(rows, m)
        for op in ("sum", "max"):
            run_and_check(gpu_lib, host, dtype, op, x_init(dtype, op, m, 11 + i), config=config)


@pytest.mark.parametrize("dtype", DTYPES)
def test_misaligned_input_uses_element_loads(gpu_lib, dtype):
    om = gpu_lib
    rows, m = 3001, 40
    flat = synth.host(dtype, rows * m + 1, 3000)
    dev = to_device(flat, dtype)[1:]
    host = flat[1:].reshape(rows, m)
    assert om.reduce_array_plan(rows, m, dtype, "sum", aligned16=False)[5] == ESIZE[dtype]
    for op in OPS:
        run_and_check(om, host, dtype, op, x_init(dtype, op, m, 5), inp=dev)


def test_two_level_groups_repeated_launches_identical(gpu_lib):
    om = gpu_lib
    rows, m = 1 << 21, 8
    plan = om.reduce_array_plan(rows, m, synth.F32, "sum", config={"teams": 4096})
    assert plan[3] > 32 and plan[4] > 1      # more than one election group
    host = synth.host(synth.F32, rows * m, 4000).reshape(rows, m)
    dev = to_device(host.reshape(-1), synth.F32)
    xh = np.zeros(m)
    first = run_and_check(om, host, synth.F32, "sum", xh, config={"teams": 4096}, inp=dev)
    s = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(s):
        for _ in range(200):
            x = torch.zeros(m, dtype=torch.float32, device="cuda")
            om.reduce_array(dev, rows, m, "sum", x, config={"teams": 4096})
            outs.append(x)
    s.synchronize()
    for x in outs:
        assert np.array_equal(x.cpu().numpy(), first)
    assert om.workspace_status(stream=s) == 0
    # int64 sums over the same groups are exact
    hi = synth.host(synth.I64, rows * m, 4001).reshape(rows, m)
    run_and_check(om, hi, synth.I64, "sum", np.zeros(m, np.int64), config={"teams": 4096})


@pytest.mark.parametrize("rows,m,cfg", [((1 << 14) + 77, 1024, {"threads": 256, "teams": 4096}),
                                        ((1 << 17) + 5, 300, {"teams": 4096})])
def test_two_level_groups_wide_rows(gpu_lib, rows, m, cfg):
    om = gpu_lib
    plan = om.reduce_array_plan(rows, m, synth.F32, "sum", config=cfg)
    assert plan[2] > 1 and plan[4] > 1       # column tiles, each with several election groups
    for dtype in (synth.F32, synth.I64):
        host = synth.host(dtype, rows * m, 4100 + m).reshape(rows, m)
        run_and_check(om, host, dtype, "sum", x_init(dtype, "sum", m, 9), config=cfg)
    assert om.workspace_status() == 0


def test_empty_and_unchanged(gpu_lib):
    om = gpu_lib
    x = torch.arange(5, dtype=torch.float32, device="cuda")
    inp = torch.ones(10, dtype=torch.float32, device="cuda")
    om.reduce_array(inp, 0, 5, "sum", x)
    om.reduce_array(inp, 2, 0, "sum", x)
    torch.cuda.synchronize()
    assert x.cpu().tolist() == [0.0, 1.0, 2.0, 3.0, 4.0]


@pytest.mark.parametrize("rows,m,dtype,op", [((1 << 25), 8, synth.F32, "sum"),
                                             ((1 << 16), 4096, synth.F32, "sum"),
                                             ((1 << 14), 1 << 14, synth.I64, "sum"),
                                             ((1 << 20), 256, synth.F32, "max")])
def test_full_size_sampled_columns(gpu_lib, rows, m, dtype, op):
    host = synth.host(dtype, rows * m, 5000).reshape(rows, m)
    cols = sorted(set([0, 1, m // 2, m - 1] + list(np.random.Generator(np.random.PCG64(1))
                                                     .integers(0, m, 12))))
    run_and_check(gpu_lib, host, dtype, op, x_init(dtype, op, m, 3), cols=cols)
