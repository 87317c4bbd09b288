"""GPU parity of maxloc / minloc against the oracle: value bits and position
exact, for every dtype on ragged sizes with many ties (small integer ranges),
under several launch configurations; planted NaNs; x_orig winning and
tying; all-NaN input; the 2^28 fp32 input in the default launch."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import TORCH_DT, to_device

pytestmark = pytest.mark.gpu

DTYPES = [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16]
SIZES = [1, 2, 63, 65, 1000, 4097, 65537, (1 << 20) | 12345]
CONFIGS = [None, {"teams": 1}, {"teams": 4096, "threads": 256, "unroll": 2}, {"unroll": 8}]


def tied_data(dtype, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    v = g.integers(-100, 100, n)
    if dtype == synth.I32:
        return v.astype(np.int32)
    if dtype == synth.I64:
        return v.astype(np.int64) * (1 << 33)
    if dtype == synth.F32:
        return (v * 0.25).astype(np.float32)
    if dtype == synth.F64:
        return (v * 0.25).astype(np.float64)
    return synth._f32_to_bf16_bits_rne((v * 0.25).astype(np.float32))


def worst(dtype, op):
    if dtype in (synth.I32, synth.I64):
        info = np.iinfo(np.int32 if dtype == synth.I32 else np.int64)
        return info.min if op == "max" else info.max
    return -np.inf if op == "max" else np.inf


def run(om, dev, dtype, op, x0, i0, config=None):
    val = torch.tensor([x0], dtype=TORCH_DT[dtype], device="cuda")
    idx = torch.tensor([i0], dtype=torch.int64, device="cuda")
    om.reduce_loc(dev, op, val, idx, config=config)
    torch.cuda.synchronize()
    v = val.float().item() if dtype == synth.BF16 else val.item()
    return v, idx.item()


def ref(host, dtype, op, x0, i0):
    xv = x0
    if dtype == synth.BF16:
        xv = float(torch.tensor([x0], dtype=torch.bfloat16).float().item())
    return oracle.reduce_loc(host, op, xv, i0, bf16=dtype == synth.BF16)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ["max", "min"])
def test_ties_and_configs(gpu_lib, dtype, op):
    for k, n in enumerate(SIZES):
        host = tied_data(dtype, n, 40 + k)
        dev = to_device(host, dtype)
        for cfg in CONFIGS:
            got = run(gpu_lib, dev, dtype, op, worst(dtype, op), -1, cfg)
            want = ref(host, dtype, op, worst(dtype, op), -1)
            assert got[1] == want[1] and got[0] == want[0], (n, cfg, got, want)


@pytest.mark.parametrize("dtype", [synth.F32, synth.F64, synth.BF16])
def test_nan_and_x_orig(gpu_lib, dtype):
    om = gpu_lib
    host = tied_data(dtype, 100003, 7)
    if dtype == synth.BF16:
        host[::7] = 0x7FC0                    # bf16 quiet NaN
    else:
        host[::7] = np.nan
    dev = to_device(host, dtype)
    for op in ("max", "min"):
        for x0, i0 in ((worst(dtype, op), -1), (100.0 if op == "max" else -100.0, 5),
                       (24.75 if op == "max" else -25.0, 0), (24.75 if op == "max" else -25.0, 10 ** 9),
                       (np.nan, 3)):
            got = run(om, dev, dtype, op, x0, i0)
            want = ref(host, dtype, op, x0, i0)
            assert got[1] == want[1] and got[0] == want[0], (op, x0, i0, got, want)
    allnan = to_device(np.full(5000, np.nan, dtype=np.float32), synth.F32) if dtype == synth.F32 else None
    if allnan is not None:
        assert run(om, allnan, synth.F32, "max", -np.inf, -1) == (-np.inf, -1)


def test_full_size_fp32(gpu_lib):
    om = gpu_lib
    n = 1 << 28
    dev = synth.device(synth.F32, n, synth.SEED_F32)
    host = dev.cpu().numpy()
    for op in ("max", "min"):
        got = run(om, dev, synth.F32, op, worst(synth.F32, op), -1)
        assert got == ref(host, synth.F32, op, worst(synth.F32, op), -1)
