"""GPU parity of the remaining OpenMP reduction identifiers (* & | ^ && ||)
against the oracle, through the plain and the array-section entry points.

Integer results and logical results are compared exactly; floating products
within 1e-6 (fp32, bf16) or (n + 2) 2^-52 (fp64, the oracle's own bound)
relative to the FP64 oracle.  Inputs: bitwise ops on full-range integers;
integer products on odd factors in [-3, 3] (the product never becomes 0, so
wrap-around is exercised) and once with a planted 0; floating products on
1 + 0.01 N(0, 1) (bf16: a balanced mix of 1 + 2^-7 and 1 - 2^-8); logical ops on non-zero data with a planted 0 (&&) or on
zeros with a planted non-zero (||).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import TORCH_DT, to_device

pytestmark = pytest.mark.gpu

INT_OPS = ["prod", "band", "bor", "bxor", "land", "lor"]
FP_OPS = ["prod", "land", "lor"]
SIZES = [1, 2, 63, 65, 1000, 4097, 65537, (1 << 20) | 12345]
CONFIGS = [None, {"teams": 1}, {"teams": 4096, "threads": 256, "unroll": 2}, {"vec": 8, "unroll": 8}]


def data(dtype, op, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    if dtype in (synth.I32, synth.I64):
        dt = np.int32 if dtype == synth.I32 else np.int64
        if op == "prod":
            a = g.choice(np.array([-3, -1, 1, 3], dtype=dt), n)
        elif op in ("band", "bor", "bxor"):
            info = np.iinfo(dt)
            a = g.integers(info.min, info.max, n, dtype=dt, endpoint=True)
            if op == "band":
                a |= dt(~0x0F0F)   # keep a few bits alive through the and-fold
        elif op == "land":
            a = g.integers(1, 100, n).astype(dt) * g.choice(np.array([-1, 1], dtype=dt), n)
        else:
            a = np.zeros(n, dtype=dt)
        return a
    v = 1.0 + 0.01 * g.standard_normal(n) if op == "prod" else g.standard_normal(n)
    if op == "lor":
        v = np.zeros(n)
    if op == "prod" and dtype == synth.BF16:
        # bf16 rounding of 1 + 0.01 N(0, 1) is biased; a shuffled multiset of
        # 1 + 2^-7 and 1 - 2^-8 in the ratio of their logarithms keeps every
        # partial product of the fold well inside the fp32 range
        a = n // 6
        b = int(round(a * np.log1p(2.0 ** -7) / -np.log1p(-(2.0 ** -8))))
        v = np.ones(n)
        v[:a] = 1.0 + 2.0 ** -7
        v[a:a + b] = 1.0 - 2.0 ** -8
        g.shuffle(v)
    if dtype == synth.F32:
        return v.astype(np.float32)
    if dtype == synth.F64:
        return v.astype(np.float64)
    return synth._f32_to_bf16_bits_rne(v.astype(np.float32))


def x_of(dtype, op, value):
    """x with the library's output type and its value as the oracle sees it."""
    if dtype == synth.BF16:
        if op == "prod":
            return torch.tensor([value], dtype=torch.float32, device="cuda"), float(value)
        t = torch.tensor([value], dtype=torch.bfloat16, device="cuda")
        return t, float(t.float().item())
    if dtype in (synth.I32, synth.I64):
        return torch.tensor([int(value)], dtype=TORCH_DT[dtype], device="cuda"), int(value)
    t = torch.tensor([value], dtype=TORCH_DT[dtype], device="cuda")
    return t, float(t.double().item())


def ref_of(host, dtype, op, x0):
    if dtype in (synth.I32, synth.I64):
        return oracle.reduce_int(host, op, x0)
    return oracle.reduce_fp(host, op, x0, bf16=dtype == synth.BF16)


def check(got, ref, dtype, op, n, what):
    if op == "prod" and dtype not in (synth.I32, synth.I64):
        tol = (n + 2) * 2.0 ** -52 if dtype == synth.F64 else 1e-6
        assert abs(got - ref) <= tol * abs(ref), (what, got, ref)
    else:
        assert got == ref, (what, got, ref)


def value(x):
    return float(x.float().item()) if x.dtype == torch.bfloat16 else x.item()


@pytest.mark.parametrize("dtype", [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16])
def test_plain_reduce_new_operators(gpu_lib, dtype):
    om = gpu_lib
    ops = INT_OPS if dtype in (synth.I32, synth.I64) else FP_OPS
    for op in ops:
        for i, n in enumerate(SIZES):
            host = data(dtype, op, n, 100 + i)
            if op == "land" and n > 3:
                host[(7 * n) // 11] = 0          # one false operand
            if op == "lor" and n > 3:
                host[(5 * n) // 13] = 1 if dtype != synth.BF16 else 0x3F80
            dev = to_device(host, dtype)
            for c, cfg in enumerate(CONFIGS):
                x0 = {"prod": 1.5 if dtype not in (synth.I32, synth.I64) else 5, "band": -1, "bor": 0,
                      "bxor": 12345, "land": 1, "lor": 0}[op]
                x, xv = x_of(dtype, op, x0)
                om.reduce(dev, op, x, config=cfg)
                torch.cuda.synchronize()
                check(value(x), ref_of(host, dtype, op, xv), dtype, op, n, (op, n, cfg))


@pytest.mark.parametrize("dtype", [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16])
def test_logical_edge_cases(gpu_lib, dtype):
    om = gpu_lib
    n = 100003
    ones = data(dtype, "land", n, 7)
    dev = to_device(ones, dtype)
    for op, x0, want in (("land", 1, 1), ("land", 0, 0), ("lor", 0, 1), ("lor", 3, 1)):
        x, xv = x_of(dtype, op, x0)
        om.reduce(dev, op, x)
        torch.cuda.synchronize()
        assert value(x) == want == ref_of(ones, dtype, op, xv)
    zeros = to_device(np.zeros(n, dtype=ones.dtype), dtype)
    for op, x0, want in (("lor", 0, 0), ("land", 1, 0)):
        x, xv = x_of(dtype, op, x0)
        om.reduce(zeros, op, x)
        torch.cuda.synchronize()
        assert value(x) == want


def test_integer_product_with_a_zero_and_nan_logic(gpu_lib):
    om = gpu_lib
    host = data(synth.I64, "prod", 70001, 3)
    host[12345] = 0
    x, _ = x_of(synth.I64, "prod", 1)
    om.reduce(to_device(host, synth.I64), "prod", x)
    torch.cuda.synchronize()
    assert x.item() == 0
    f = np.ones(1000, dtype=np.float32)
    f[500] = np.nan                      # NaN is a true operand
    x, _ = x_of(synth.F32, "land", 1.0)
    om.reduce(to_device(f, synth.F32), "land", x)
    torch.cuda.synchronize()
    assert x.item() == 1.0


@pytest.mark.parametrize("dtype", [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16])
def test_array_section_new_operators(gpu_lib, dtype):
    om = gpu_lib
    ops = INT_OPS if dtype in (synth.I32, synth.I64) else FP_OPS
    for op in ops:
        for j, (rows, m) in enumerate([(1000, 3), (2049, 64), (300, 257), (64, 4096), (20000, 1)]):
            host = data(dtype, op, rows * m, 300 + j).reshape(rows, m)
            if op == "land":
                host[(3 * rows) // 7, ::3] = 0
            if op == "lor":
                host[(2 * rows) // 5, ::2] = 1 if dtype != synth.BF16 else 0x3F80
            dev = to_device(host.reshape(-1), dtype)
            x0 = {"prod": 1.0 if dtype not in (synth.I32, synth.I64) else 1, "band": -1, "bor": 0,
                  "bxor": 0, "land": 1, "lor": 0}[op]
            if dtype == synth.BF16 and op == "prod":
                x = torch.full((m,), x0, dtype=torch.float32, device="cuda")
            elif dtype in (synth.I32, synth.I64):
                x = torch.full((m,), x0, dtype=TORCH_DT[dtype], device="cuda")
            else:
                x = torch.full((m,), float(x0), dtype=TORCH_DT[dtype], device="cuda")
            for cfg in (None, {"teams": 2048}):
                xx = x.clone()
                om.reduce_array(dev, rows, m, op, xx, config=cfg)
                torch.cuda.synchronize()
                got = xx.float().cpu().numpy().astype(np.float64) if xx.dtype == torch.bfloat16 \
                    else xx.cpu().numpy()
                for col in range(m):
                    ref = ref_of(np.ascontiguousarray(host[:, col]), dtype, op, x0)
                    check(got[col].item(), ref, dtype, op, rows, (op, rows, m, col, cfg))
