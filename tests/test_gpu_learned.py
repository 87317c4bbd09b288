"""The learned launch-configuration picker on the GPU.

* With the trained model loaded, reductions and AXPY bodies whose launch the
  model picks still match the oracle (bit-exact integers / y, 1e-6 sums).
* The model's picks beat the built-in heuristic on held-out instances
  (total time over a sample of the held-out distribution), which is what
  the trained network gains over the method without it.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check_axpy, check_value, identity, oracle_value, to_device, x_tensor, x_value

pytestmark = pytest.mark.gpu

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2106_03219_amd", "picker_model.txt")
OPN = {0: "sum", 1: "max", 2: "min"}


@pytest.fixture
def model(gpu_lib):
    if not os.path.exists(MODEL):
        pytest.skip("no trained model file in the package")
    gpu_lib.model_load(MODEL)
    yield gpu_lib
    gpu_lib.model_load(None)


def test_model_picked_launches_match_oracle(model):
    om = model
    inst = synth.cost_instances(60, 1234, 3.0, 6.5)
    picked = 0
    for i in range(60):
        n, dt, op, body, ch = (int(inst[k][i]) for k in ("n", "dtype", "op", "body", "chunk"))
        _, src = om.resolve_config(n, dt, op, body, ch)
        picked += src == 1
        if body:
            x = synth.f32_normal(n, 500 + i)
            y = synth.f32_normal(n, 900 + i)
            xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
            s = torch.zeros(1, dtype=torch.float32, device="cuda")
            om.axpy_sum(0.7, xd, yd, s, 0, 0, 0, max(ch, 0))
            torch.cuda.synchronize()
            y_ref, s_ref = oracle.axpy_sum(0.7, x, y)
            check_axpy(yd.cpu().numpy(), s.item(), y_ref, s_ref, 0.0, (n, ch))
        else:
            host = synth.host(dt, n, 700 + i)
            xo = x_tensor(dt, OPN[op], identity(dt, OPN[op]))
            om.reduce(to_device(host, dt), OPN[op], xo)
            torch.cuda.synchronize()
            ref, sabs = oracle_value(host, dt, OPN[op], identity(dt, OPN[op]))
            check_value(x_value(xo), ref, sabs, dt, OPN[op], f"instance {i}")
    assert picked > 0


def _total_time(om, insts, bufs, use_model):
    cfg = None if use_model else {"flags": om.CFG_NO_MODEL}
    total = 0.0
    for n, dt, op, body, ch in insts:
        if body:
            x, y = bufs[synth.F32][:n], bufs["y"][:n]
            s = torch.zeros(1, dtype=torch.float32, device="cuda")
            fn = lambda: om.axpy_sum(0.7, x, y, s, 0, 0, 0, max(ch, 0), config=cfg)
        else:
            inp = bufs[dt][:n]
            xo = x_tensor(dt, OPN[op], identity(dt, OPN[op]))
            fn = lambda: om.reduce(inp, OPN[op], xo, config=cfg)
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        total += min(a.elapsed_time(b) for a, b in evs)
    return total


def test_model_beats_heuristic_on_heldout_sample(model):
    om = model
    inst = synth.cost_instances(400, synth.SEED_HELDOUT)
    keep = [i for i in range(400) if inst["n"][i] <= 10**8][:300]
    insts = [tuple(int(inst[k][i]) for k in ("n", "dtype", "op", "body", "chunk")) for i in keep]
    nmax = max(t[0] for t in insts)
    bufs = {dt: synth.device(dt, nmax, 40 + dt) for dt in (synth.I32, synth.I64, synth.F32, synth.BF16)}
    bufs["y"] = synth.device(synth.F32, nmax, 50)
    t_model = _total_time(om, insts, bufs, True)
    t_heur = _total_time(om, insts, bufs, False)
    print(f"held-out sample: model {t_model:.2f} ms, heuristic {t_heur:.2f} ms")
    assert t_model < t_heur
