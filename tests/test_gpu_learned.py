"""The learned launch-configuration picker on the GPU.

* With the trained model loaded, reductions and AXPY bodies whose launch the
  model picks still match the oracle (bit-exact integers / y, 1e-6 sums).
* The model's picks beat the built-in heuristic on held-out instances
  (total time over a sample of the held-out distribution, timed as the
  autotuner times: the GPU time a launch adds to a stream of launches over
  inputs not in cache), which is what the trained network gains over the
  method without it.
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


def _total_time(om, insts, bufs, nmax, use_model):
    """Total over the instances of the GPU time a launch adds to a stream of launches over
    uncached inputs -- the autotuner's own measure (tune.time_call with rotating windows)."""
    from paper_2106_03219_amd.tune import Windows, calibrate_spin, time_call
    calibrate_spin(torch)
    cursor = [0]
    cfg = None if use_model else {"flags": om.CFG_NO_MODEL}
    total = 0.0
    for n, dt, op, body, ch in insts:
        eb = 12 if body else {synth.I32: 4, synth.I64: 8, synth.F32: 4, synth.BF16: 2}[dt]
        win = Windows(cursor, n, nmax, 3 if n * eb > (64 << 20) else 8)
        if body:
            xb, yb = bufs[synth.F32], bufs["y"]
            s = torch.zeros(1, dtype=torch.float32, device="cuda")
            fn = lambda o: om.axpy_sum(0.7, xb[o:o + n], yb[o:o + n], s, 0, 0, 0, max(ch, 0),
                                       config=cfg)
        else:
            full = bufs[dt]
            xo = x_tensor(dt, OPN[op], identity(dt, OPN[op]))
            fn = lambda o: om.reduce(full[o:o + n], OPN[op], xo, config=cfg)
        total += time_call(fn, 2, torch, win) / 1e3
    return total


def test_model_beats_heuristic_on_heldout_sample(model):
    om = model
    inst = synth.cost_instances(400, synth.SEED_HELDOUT)
    keep = [i for i in range(400) if inst["n"][i] <= 10**8][:300]
    insts = [tuple(int(inst[k][i]) for k in ("n", "dtype", "op", "body", "chunk")) for i in keep]
    nmax = max(t[0] for t in insts)
    bufs = {dt: synth.device(dt, nmax, 40 + dt) for dt in (synth.I32, synth.I64, synth.F32, synth.BF16)}
    bufs["y"] = synth.device(synth.F32, nmax, 50)
    t_model = _total_time(om, insts, bufs, nmax, True)
    t_heur = _total_time(om, insts, bufs, nmax, False)
    print(f"held-out sample: model {t_model:.2f} ms, heuristic {t_heur:.2f} ms")
    assert t_model < t_heur
