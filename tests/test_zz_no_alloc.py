"""GPU parity of omprt_reduce_noalloc (cross-team state in a fixed device
array, no allocation) against omprt_reduce, both called through the C ABI on
the same inputs: integers, max and min bit for bit, fp32 / bf16 / fp64 sums to
the sum tolerance (and both against the oracle).  Every case makes two calls
in a row, the second over a smaller input with fewer teams, so the second
runs on the state the first left in the array.  Beyond 4096 teams the call
is refused.
"""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_util import (OPS, check_value, identity, oracle_value, to_device, to_host,
                      x_tensor, x_value)

pytestmark = pytest.mark.gpu


def _cfg(om, c):
    if not c:
        return None
    return ctypes.byref(om.Config(c.get("teams", 0), c.get("threads", 0), 0, 0, 0,
                                  c.get("flags", 0)))


def _call(om, name, dev, dtype, op, x0, cfg):
    """One call of the entry point `name` through the C ABI; x after the call."""
    lib = om.load()
    x = x_tensor(dtype, op, x0)
    st = getattr(lib, name)(ctypes.c_void_p(dev.data_ptr()), dev.numel(), dtype,
                            om._op(op), ctypes.c_void_p(x.data_ptr()), _cfg(om, cfg), None)
    assert st == 0, (name, st, lib.omprt_last_error())
    torch.cuda.synchronize()
    return x_value(x)


# (n of the first call, its config), (n of the second, smaller, call, its config)
PAIRS = [
    (((1 << 22) + 7, {}), (100003, {})),
    (((1 << 21) + 3, {"teams": 4096, "threads": 256}), (65537, {"teams": 7, "threads": 64})),
    ((1000003, {"teams": 300, "threads": 1024}), (4099, {"teams": 2, "threads": 128})),
    ((1 << 20, {"teams": 64, "threads": 512, "flags": 0x10}),
     (50001, {"teams": 3, "threads": 256, "flags": 0x10})),
]


@pytest.mark.parametrize("dtype", [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16])
@pytest.mark.parametrize("pair", range(len(PAIRS)))
def test_noalloc_matches_reduce_two_calls(gpu_lib, dtype, pair):
    om = gpu_lib
    for k, (n, cfg) in enumerate(PAIRS[pair]):
        host = synth.host(dtype, n, 700 + 10 * pair + k)
        dev = to_device(host, dtype)
        for op in OPS:
            x0 = identity(dtype, op) if op != "sum" else (3 if dtype in (synth.I32, synth.I64)
                                                          else 1.5)
            got = _call(om, "omprt_reduce_noalloc", dev, dtype, op, x0, cfg)
            ref_call = _call(om, "omprt_reduce", dev, dtype, op, x0, cfg)
            ref, sabs = oracle_value(host, dtype, op, x0)
            what = (n, op, cfg)
            check_value(got, ref, sabs, dtype, op, f"noalloc {what}", n=n)
            check_value(ref_call, ref, sabs, dtype, op, f"reduce {what}", n=n)
            if dtype in (synth.I32, synth.I64) or op != "sum":
                assert got == ref_call, what
            else:
                tol = 2e-12 if dtype == synth.F64 else 2e-6
                bound = tol * abs(ref) if ref != 0 else tol * sabs
                assert abs(got - ref_call) <= bound, (what, got, ref_call)


def test_noalloc_empty_and_limits(gpu_lib):
    om = gpu_lib
    lib = om.load()
    dev = to_device(synth.host(synth.I32, 10000, 5), synth.I32)
    x = torch.tensor([42], dtype=torch.int32, device="cuda")
    assert lib.omprt_reduce_noalloc(ctypes.c_void_p(dev.data_ptr()), 0, synth.I32, om._op("sum"),
                                    ctypes.c_void_p(x.data_ptr()), None, None) == 0
    torch.cuda.synchronize()
    assert int(x.item()) == 42
    st = lib.omprt_reduce_noalloc(ctypes.c_void_p(dev.data_ptr()), dev.numel(), synth.I32,
                                  om._op("sum"), ctypes.c_void_p(x.data_ptr()),
                                  _cfg(om, {"teams": 4097, "threads": 64}), None)
    assert st == 1   # OMPRT_ERR_INVALID
    assert b"4096" in lib.omprt_last_error()
    # the array is still healthy after the refused call
    host = to_host(dev)
    got = _call(om, "omprt_reduce_noalloc", dev, synth.I32, "sum", 0,
                {"teams": 4096, "threads": 64})
    assert got == int(host.astype(np.int64).sum())
