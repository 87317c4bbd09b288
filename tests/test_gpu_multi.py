"""GPU parity of several reduction variables over one input in one pass
(reduction(+: s) reduction(max: hi) reduction(min: lo)): every subset of
{sum, max, min} in any order, every dtype, ragged sizes and several launch
configurations, x_orig != identity; each variable against the oracle's
scalar fold (gpu_util tolerances), and against a separate omprt_reduce of
the same op (integers, max and min bit-identical)."""
import itertools

import numpy as np
import pytest
import torch

import synth
from gpu_util import check_value, oracle_value, to_device, x_tensor, x_value

pytestmark = pytest.mark.gpu

DTYPES = [synth.I32, synth.I64, synth.F32, synth.F64, synth.BF16]
SUBSETS = [c for k in (1, 2, 3) for c in itertools.permutations(("sum", "max", "min"), k)]
SIZES = [1, 63, 65, 4097, 65537, (1 << 20) | 12345]
CONFIGS = [None, {"teams": 1}, {"teams": 4096, "threads": 256, "unroll": 2}]
X0 = {"sum": 3, "max": 0, "min": 0}


@pytest.mark.parametrize("dtype", DTYPES)
def test_subsets_sizes_configs(gpu_lib, dtype):
    om = gpu_lib
    for k, n in enumerate(SIZES):
        host = synth.host(dtype, n, 600 + k)
        dev = to_device(host, dtype)
        for cfg in CONFIGS:
            for ops in SUBSETS:
                xs = [x_tensor(dtype, op, X0[op]) for op in ops]
                om.reduce_multi(dev, list(zip(ops, xs)), config=cfg)
                torch.cuda.synchronize()
                for op, x in zip(ops, xs):
                    x0v = x_value(x_tensor(dtype, op, X0[op]))
                    ref, sabs = oracle_value(host, dtype, op, x0v)
                    check_value(x_value(x), ref, sabs, dtype, op, (n, cfg, ops, op))
                    if op != "sum" or dtype in (synth.I32, synth.I64):
                        single = x_tensor(dtype, op, X0[op])
                        om.reduce(dev, op, single, config=cfg)
                        torch.cuda.synchronize()
                        assert x_value(single) == x_value(x)


def test_full_size_statistics_fp32(gpu_lib):
    om = gpu_lib
    n = 1 << 28
    dev = synth.device(synth.F32, n, synth.SEED_F32)
    host = dev.cpu().numpy()
    xs = {op: x_tensor(synth.F32, op, 0 if op == "sum" else (-np.inf if op == "max" else np.inf))
          for op in ("sum", "max", "min")}
    om.reduce_multi(dev, list(xs.items()))
    torch.cuda.synchronize()
    for op, x in xs.items():
        x0 = 0.0 if op == "sum" else (-np.inf if op == "max" else np.inf)
        ref, sabs = oracle_value(host, synth.F32, op, x0)
        check_value(x_value(x), ref, sabs, synth.F32, op, op)


def test_argument_errors(gpu_lib):
    om = gpu_lib
    dev = torch.ones(10, device="cuda")
    x = torch.zeros(1, device="cuda")
    with pytest.raises(om.OmprtError):
        om.reduce_multi(dev, [("sum", x), ("sum", x)])
    with pytest.raises(om.OmprtError):
        om.reduce_multi(dev, [("prod", x)])
    with pytest.raises(om.OmprtError):
        om.reduce_multi(dev, [("sum", x)], config={"unroll": 8})
