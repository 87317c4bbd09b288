"""GPU parity of user-defined reductions (declare reduction, compiled at run
time) against the oracle's sequential fold of the same reduction:

* exact types (STATS3 over int32, MINMAX over fp64, HIST16 over int64, 64
  bytes: four cross-team slots): bit-exact, also with an original value that
  is not the identity;
* WELFORD over fp32 and bf16: count exact; mean within 1e-12 (|mean| + sd)
  and M2 within 1e-10 relative of the moments' definitions -- double
  arithmetic, a different but stable combination order;
* SUMSQ over bf16: within 1e-11 relative (double sums of at most 2^21 exact
  squares in another order: typical error sqrt(n) u ~ 1e-13);
* ragged sizes, n = 0 (x unchanged), one team, many small teams, and 2^24
  fp32 in the default launch (the oracle's exactly rounded sums bound the
  size).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import udr_cases as U
from gpu_util import to_device

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 65, 1000, 4097, 65537, (1 << 20) | 12345]
CONFIGS = [None, {"teams": 1}, {"teams": 4096, "threads": 64}, {"teams": 300, "threads": 1024}]


def declare(om, name, dtype):
    c = getattr(U, name)
    return om.udr_declare(c["type_def"], c["initializer"], c["combiner"], c["body"], c["acc_bytes"],
                          dtype)


def run(om, h, name, dev, x0, config=None):
    x = torch.from_numpy(U.pack(name, x0)).cuda()
    om.reduce_udr(h, dev, x, config=config)
    torch.cuda.synchronize()
    assert om.workspace_status() == 0
    return U.unpack(name, x.cpu().numpy())


def fold(name, host, x0):
    f = name.lower()
    return oracle.udr_fold(host, x0, getattr(U, f + "_init"), getattr(U, f + "_body"),
                           getattr(U, f + "_combine"))


@pytest.mark.parametrize("name,dtype,gen", [
    ("STATS3", synth.I32, lambda n, s: synth.int32_uniform(n, s, lo=-(2 ** 31), hi=2 ** 31 - 1)),
    ("MINMAX", synth.F64, lambda n, s: np.round(synth.f64_normal(n, s) * 8) / 8),   # many ties
    ("HIST16", synth.I64, synth.int64_uniform),
])
def test_exact_types(gpu_lib, name, dtype, gen):
    h = declare(gpu_lib, name, dtype)
    ident = getattr(U, name.lower() + "_init")()
    for k, n in enumerate(SIZES):
        host = gen(n, 500 + k)
        dev = to_device(host, dtype)
        want = fold(name, host.tolist(), ident)
        for cfg in CONFIGS:
            got = run(gpu_lib, h, name, dev, ident, cfg)
            assert got == want, (name, n, cfg, got, want)
    # an original value that is not the identity takes part through the combiner
    host = gen(10007, 77)
    x0 = {"STATS3": (5, 7, 11), "MINMAX": (-1e300, 1e300, 3, 0), "HIST16": tuple(range(16))}[name]
    assert run(gpu_lib, h, name, to_device(host, dtype), x0) == fold(name, host.tolist(), x0)


def _check_moments(got, ref):
    n, mean, m2 = ref
    assert got[0] == n
    sd = (m2 / n) ** 0.5 if n else 0.0
    assert abs(got[1] - mean) <= 1e-12 * (abs(mean) + sd), (got, ref)
    assert abs(got[2] - m2) <= 1e-10 * m2 + 1e-300, (got, ref)


@pytest.mark.parametrize("dtype", [synth.F32, synth.BF16])
def test_welford(gpu_lib, dtype):
    h = declare(gpu_lib, "WELFORD", dtype)
    for k, n in enumerate(SIZES):
        host = synth.host(dtype, n, 600 + k)
        if dtype == synth.F32:
            host = (host * 3 + 50).astype(np.float32)      # mean far from zero
            wide = host.astype(np.float64)
        else:
            wide = (host.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        dev = to_device(host, dtype)
        ref = oracle.moments(wide)
        for cfg in CONFIGS:
            _check_moments(run(gpu_lib, h, "WELFORD", dev, U.welford_init(), cfg), ref)


def test_sumsq_bf16(gpu_lib):
    h = declare(gpu_lib, "SUMSQ", synth.BF16)
    for k, n in enumerate(SIZES):
        host = synth.host(synth.BF16, n, 700 + k)
        wide = (host.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        ref = fold("SUMSQ", wide.tolist(), (0.0,))[0]
        for cfg in CONFIGS:
            got = run(gpu_lib, h, "SUMSQ", to_device(host, synth.BF16), (0.0,), cfg)[0]
            assert abs(got - ref) <= 1e-11 * ref, (n, cfg, got, ref)


def test_empty_input_leaves_x(gpu_lib):
    h = declare(gpu_lib, "STATS3", synth.I32)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert run(gpu_lib, h, "STATS3", empty, (1, 2, 3)) == (1, 2, 3)


def test_welford_2pow24_default_launch(gpu_lib):
    n = 1 << 24
    h = declare(gpu_lib, "WELFORD", synth.F32)
    dev = synth.device(synth.F32, n, synth.SEED_F32)
    got = run(gpu_lib, h, "WELFORD", dev, U.welford_init())
    _check_moments(got, oracle.moments(dev.cpu().numpy().astype(np.float64)))
