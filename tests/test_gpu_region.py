"""GPU parity of the two-loop region (AXPY loop [nowait], then a sum loop)
against the oracle: y bit-exact (fused multiply-add on both sides), sum
within 1e-6 of the FP64 sum of the updated y -- the same results as the
fused body.  Schedules: ragged sizes, teams x threads (also not multiples of
64), distribute chunks, chunks 0 / 1 / 7 / 64 / 1024, nowait with equal
chunks, the barrier with equal and with different chunks (loop 2 then reads
elements other threads wrote), x / y misalignment, and 2^26 elements.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check_axpy

pytestmark = pytest.mark.gpu
A = 0.7


def _run(om, x_h, y_h, teams, threads, dc, c1, c2, nowait, s0=0.0, xoff=0, yoff=0):
    n = x_h.size
    xd = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
    yd = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
    xd[xoff:xoff + n] = torch.from_numpy(x_h).cuda()
    yd[yoff:yoff + n] = torch.from_numpy(y_h).cuda()
    s = torch.tensor([s0], dtype=torch.float32, device="cuda")
    om.region_axpy_sum(A, xd[xoff:xoff + n], yd[yoff:yoff + n], s, teams, threads, dc, c1, c2, nowait)
    torch.cuda.synchronize()
    y_ref, s_ref = oracle.axpy_sum(A, x_h, y_h, s0)
    case = (n, teams, threads, dc, c1, c2, nowait)
    check_axpy(yd[yoff:yoff + n].cpu().numpy(), s.item(), y_ref, s_ref, s0, case)
    assert om.workspace_status() == 0, case


SCHEDS = [(1, 1, 1, 0), (100, 2, 64, 0), (1000, 3, 9, 0), (1000, 3, 9, 13), (4099, 5, 100, 0),
          (65537, 16, 256, 0), (65537, 16, 256, 1000), (100003, 128, 64, 0), (100003, 0, 0, 0),
          (5, 8, 64, 0), (300001, 7, 1000, 0),
          # whole-wave teams with lane runs of one line or more (through LDS
          # lines): aligned and ragged runs, distribute blocks
          ((1 << 20) + 3, 4, 256, 0), (300000, 7, 512, 0), ((1 << 20) + 37, 3, 192, 5000),
          # the runtime's own launch (its chunk-dependent choices) at a larger size
          ((1 << 21) + 11, 0, 0, 0)]


@pytest.mark.parametrize("n,T,P,dc", SCHEDS)
@pytest.mark.parametrize("c", [0, 1, 7, 16, 32, 64, 544, 1024])
def test_nowait_and_barrier_same_schedule(gpu_lib, n, T, P, dc, c):
    x = synth.f32_normal(n, 50 + n)
    y = synth.f32_normal(n, 51 + n)
    for nowait in (True, False):
        _run(gpu_lib, x, y, T, P, dc, c, c, nowait, s0=1.25)


@pytest.mark.parametrize("c1,c2", [(0, 1), (1, 0), (7, 64), (1024, 1), (64, 0)])
def test_barrier_different_schedules(gpu_lib, c1, c2):
    for k, (n, T, P, dc) in enumerate(SCHEDS):
        x = synth.f32_normal(n, 60 + k)
        y = synth.f32_normal(n, 61 + k)
        _run(gpu_lib, x, y, T, P, dc, c1, c2, False)


def test_misaligned(gpu_lib):
    x = synth.f32_normal(50001, 3)
    y = synth.f32_normal(50001, 4)
    # (1, 2) and (3, 0): x and y not co-aligned; (2, 2) and (4, 0): co-aligned
    # to 16 bytes, with line boundaries inside the runs
    for xo, yo in [(1, 1), (1, 2), (3, 0), (2, 2), (4, 0)]:
        for c in (0, 1, 64):
            _run(gpu_lib, x, y, 8, 256, 0, c, c, True, xoff=xo, yoff=yo)
        _run(gpu_lib, x, y, 8, 256, 0, 0, 64, False, xoff=xo, yoff=yo)


@pytest.mark.parametrize("c", [0, 1, 64])
def test_2pow26(gpu_lib, c):
    n = 1 << 26
    x = synth.f32_normal(n, synth.SEED_AXPY_X)
    y = synth.f32_normal(n, synth.SEED_AXPY_Y)
    _run(gpu_lib, x, y, 0, 0, 0, c, c, True)
    _run(gpu_lib, x, y, 0, 0, 0, c, c, False)
