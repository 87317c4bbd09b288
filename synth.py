"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers: it holds none of the reductions,
schedules or model arithmetic, so neither the HIP path nor the CPU oracle
depends on the other through it.  Host arrays come from numpy's PCG64;
large device-resident inputs come from torch's seeded device generator
(Philox) and are copied back to the host when the oracle needs them.

Workload shapes (sizes, distributions) follow the data-parallel core's
benchmark configurations: int32 uniform in [-1000, 1000]; fp32 ~ N(0, 1);
int64 uniform in [-2^40, 2^40]; bf16 = round-to-nearest-even of N(0, 1);
segment lengths log-uniform in [1e2, 1e7]; cost-model instances with
N log-uniform in [1e3, 1e9].
"""
from __future__ import annotations

import numpy as np

# dtype / op codes shared by both sides' call conventions (plain integers)
I32, I64, F32, F64, BF16 = 0, 1, 2, 3, 4
SUM, MAX, MIN = 0, 1, 2
NP_DTYPE = {I32: np.int32, I64: np.int64, F32: np.float32, F64: np.float64, BF16: np.uint16}
ELEM_BYTES = {I32: 4, I64: 8, F32: 4, F64: 8, BF16: 2}

SEED_C1, SEED_F32, SEED_I64, SEED_AXPY_X, SEED_AXPY_Y, SEED_BATCH = 1, 2, 3, 4, 5, 6
SEED_TRAIN, SEED_HELDOUT = 7, 8


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def int32_uniform(n: int, seed: int, lo: int = -1000, hi: int = 1000) -> np.ndarray:
    """int32 uniform on [lo, hi] inclusive."""
    return rng(seed).integers(lo, hi, size=n, endpoint=True, dtype=np.int32)


def int64_uniform(n: int, seed: int, lo: int = -(2**40), hi: int = 2**40) -> np.ndarray:
    return rng(seed).integers(lo, hi, size=n, endpoint=True, dtype=np.int64)


def f32_normal(n: int, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(n, dtype=np.float32)


def f64_normal(n: int, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(n, dtype=np.float64)


def power_inputs(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Diagonal and start vector for the power iteration (fp32): d has a
    random sign and magnitude uniform on [0.75, 1] (after 100 steps a
    component has shrunk by at most 0.75^100 ~ 3e-13 against the largest,
    far from fp32 underflow), v0 is standard normal."""
    g = rng(seed)
    d = (g.uniform(0.75, 1.0, n) * g.choice([-1.0, 1.0], n)).astype(np.float32)
    return d, g.standard_normal(n, dtype=np.float32)


def _f32_to_bf16_bits_rne(f: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns of finite fp32 values, round to nearest even."""
    u = f.view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


def bf16_normal(n: int, seed: int) -> np.ndarray:
    """bf16 bits (uint16) of RNE(N(0,1))."""
    return _f32_to_bf16_bits_rne(f32_normal(n, seed))


def host(dtype: int, n: int, seed: int) -> np.ndarray:
    """The standard distribution of each dtype, on the host."""
    if dtype == I32:
        return int32_uniform(n, seed)
    if dtype == I64:
        return int64_uniform(n, seed)
    if dtype == F32:
        return f32_normal(n, seed)
    if dtype == F64:
        return f64_normal(n, seed)
    if dtype == BF16:
        return bf16_normal(n, seed)
    raise ValueError(dtype)


# ---------------------------------------------------------------- device side

def device(dtype: int, n: int, seed: int, dev: str = "cuda"):
    """The same distributions drawn directly on the GPU with a seeded torch generator.

    Returns a torch tensor (bf16 as torch.bfloat16).  Used for inputs too large
    to draw on the host in reasonable time; the oracle reads a host copy.
    """
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    if dtype == I32:
        return torch.randint(-1000, 1001, (n,), generator=g, device=dev, dtype=torch.int32)
    if dtype == I64:
        return torch.randint(-(2**40), 2**40 + 1, (n,), generator=g, device=dev, dtype=torch.int64)
    if dtype == F32:
        return torch.randn(n, generator=g, device=dev, dtype=torch.float32)
    if dtype == F64:
        return torch.randn(n, generator=g, device=dev, dtype=torch.float64)
    if dtype == BF16:
        return torch.randn(n, generator=g, device=dev, dtype=torch.float32).to(torch.bfloat16)
    raise ValueError(dtype)


# ---------------------------------------------------------------- batched workload

def batched_spec(count: int = 4096, seed: int = SEED_BATCH, lo_exp: float = 2.0,
                 hi_exp: float = 7.0, dtypes=(I64, F32, BF16), ops=(SUM, MAX, MIN)):
    """Segment lengths floor(10^U[lo_exp, hi_exp]), dtype and op uniform over the lists."""
    g = rng(seed)
    lens = np.floor(10.0 ** g.uniform(lo_exp, hi_exp, count)).astype(np.int64)
    dts = np.asarray(dtypes)[g.integers(0, len(dtypes), count)]
    opv = np.asarray(ops)[g.integers(0, len(ops), count)]
    return lens, dts.astype(np.int32), opv.astype(np.int32)


# ---------------------------------------------------------------- cost-model instances

def cost_instances(count: int, seed: int, lo_exp: float = 3.0, hi_exp: float = 9.0):
    """Random reduction / AXPY instances for the learned configuration picker.

    Returns a dict of arrays: n (log-uniform), dtype in {i32, i64, f32, bf16},
    op in {sum, max, min}, body in {0 = none, 1 = AXPY}, chunk (-1 = no user
    chunk; otherwise one of 0, 1, 64, 1024, only for AXPY bodies).
    """
    g = rng(seed)
    n = np.floor(10.0 ** g.uniform(lo_exp, hi_exp, count)).astype(np.int64)
    dt = np.array([I32, I64, F32, BF16])[g.integers(0, 4, count)]
    op = np.array([SUM, MAX, MIN])[g.integers(0, 3, count)]
    body = g.integers(0, 2, count)
    ch = np.array([-1, 0, 1, 64, 1024])[g.integers(0, 5, count)]
    ch = np.where(body == 1, ch, -1)
    # the AXPY body is fp32 only, sum only
    dt = np.where(body == 1, F32, dt)
    op = np.where(body == 1, SUM, op)
    return {"n": n, "dtype": dt.astype(np.int32), "op": op.astype(np.int32),
            "body": body.astype(np.int32), "chunk": ch.astype(np.int64)}
