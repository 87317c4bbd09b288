"""GPU parity of the AXPY worksharing body (exact static mapping) against
the oracle: y bit-exact (fused multiply-add on both sides), sum within
1e-6 of the FP64 sum of the updated y.  Ragged and chunked schedules, the
2^26 element configuration over chunk {default, 1, 64, 1024} x teams
{64, 128, ..., 4096}, and x/y misalignment.  y' and its sum do not depend on
the schedule, so the oracle runs once per input.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check_axpy

pytestmark = pytest.mark.gpu
A = 0.7


def _run(om, x_h, y_h, teams, threads, dc, c, s0=0.0, xoff=0, yoff=0, config=None, ref=None):
    n = x_h.size
    xd = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
    yd = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
    xd[xoff:xoff + n] = torch.from_numpy(x_h).cuda()
    yd[yoff:yoff + n] = torch.from_numpy(y_h).cuda()
    s = torch.tensor([s0], dtype=torch.float32, device="cuda")
    om.axpy_sum(A, xd[xoff:xoff + n], yd[yoff:yoff + n], s, teams, threads, dc, c, config=config)
    torch.cuda.synchronize()
    y_ref, s_ref = ref if ref is not None else oracle.axpy_sum(A, x_h, y_h, s0)
    check_axpy(yd[yoff:yoff + n].cpu().numpy(), s.item(), y_ref, s_ref, s0,
               (n, teams, threads, dc, c))


SMALL = [(1, 1, 1, 0, 0), (100, 2, 64, 0, 0), (1000, 3, 9, 0, 1), (1000, 3, 9, 13, 5),
         (4099, 5, 100, 0, 7), (65537, 16, 256, 0, 64), (65537, 16, 256, 1000, 1024),
         (100003, 128, 64, 0, 0), (100003, 0, 0, 0, 0), (5, 8, 64, 0, 0),
         # whole-wave teams with lane runs (chunk 0 or >= 64): lines through LDS,
         # with ragged runs (heads and tails per lane), short runs (no whole
         # line), dist_schedule blocks, a final partial round of chunks
         (300000, 7, 256, 0, 0), (300000, 7, 512, 0, 100), ((1 << 20), 4, 128, 0, 0),
         ((1 << 20) + 37, 3, 192, 5000, 64), (1000, 2, 256, 0, 0), (70000, 1, 512, 0, 2048),
         ((1 << 20) + 5, 9, 448, 0, 96), (200000, 33, 64, 0, 0),
         # the runtime's own launch for the chunk sizes it treats apart (chunk 1:
         # one team of 512 per compute unit; 1024 and more: 512 threads, ~128
         # chunks a team), ragged sizes
         (100003, 0, 0, 0, 1), (300001, 0, 0, 0, 1024), (1000003, 0, 0, 0, 4096),
         (70000, 0, 0, 0, 4096),
         # chunks over 512 at the runtime's own launch: a team per wave of chunks (64
         # threads; 128 with 300 waves of chunks), and 512 threads with the team count
         # rounded down to whole rounds (33 001 chunks of 768: 258 -> 256 teams)
         ((1 << 21) + 3, 0, 0, 0, 768), (11_520_007, 0, 0, 0, 600), (25_344_005, 0, 0, 0, 768),
         # short runs off the line grid through the union of a wave's runs:
         # chunks 16 to 128, chunk 0 shares of up to 128, a final partial round
         (200003, 8, 256, 0, 16), (200003, 8, 256, 0, 32), ((1 << 20) + 5, 32, 256, 0, 120),
         (1000003, 64, 256, 0, 0), (1000003, 512, 64, 0, 0), (333333, 3, 128, 0, 48),
         ((1 << 20), 4, 256, 0, 16), ((1 << 20) + 64, 4, 256, 0, 32),
         # chunks of 8 to 15 with team blocks off the line grid (the union), and 7 (lane by lane)
         ((1 << 20) + 5, 8, 256, 0, 8), (300001, 7, 192, 0, 12), ((1 << 20) + 3, 0, 0, 0, 15),
         (200003, 3, 64, 0, 7)]


@pytest.mark.parametrize("n,T,P,dc,c", SMALL)
def test_axpy_small_schedules(gpu_lib, n, T, P, dc, c):
    x = synth.f32_normal(n, 40 + n)
    y = synth.f32_normal(n, 41 + n)
    _run(gpu_lib, x, y, T, P, dc, c, s0=1.25)


# Lane runs of 15 to 128 lines; from 16 lines on a wave takes its lines in a
# rotated order that depends on the wave (so many teams give many starting
# lines): chunks around that threshold, chunk-0 shares of 16, 17 and 100
# lines a lane, ragged ends; each run again with x and y one element off the
# line grid (a head before the first line, one line fewer).
ROTATED = [(64 * 64 * 480 + 5, 64, 64, 0, 480), (37 * 64 * 512, 37, 64, 0, 512),
           (37 * 64 * 544 + 3, 37, 64, 0, 544), (23 * 128 * 1056, 23, 128, 0, 1056),
           (9 * 64 * 4096 + 77, 9, 64, 0, 4096), (41 * 256 * 512, 41, 256, 0, 0),
           (41 * 256 * 544 + 100, 41, 256, 0, 0), (13 * 192 * 3200, 13, 192, 0, 0)]


@pytest.mark.parametrize("n,T,P,dc,c", ROTATED)
def test_axpy_rotated_lines(gpu_lib, n, T, P, dc, c):
    x = synth.f32_normal(n, 70 + n % 1000)
    y = synth.f32_normal(n, 71 + n % 1000)
    ref = oracle.axpy_sum(A, x, y, 0.5)
    _run(gpu_lib, x, y, T, P, dc, c, s0=0.5, ref=ref)
    _run(gpu_lib, x, y, T, P, dc, c, s0=0.5, xoff=1, yoff=1, ref=ref)


def test_axpy_misaligned(gpu_lib):
    x = synth.f32_normal(50001, 3)
    y = synth.f32_normal(50001, 4)
    # (1, 2) and (3, 0): x and y not co-aligned; (2, 2) and (4, 0): co-aligned
    # to 16 bytes, with line boundaries inside the runs
    for xo, yo in [(1, 1), (1, 2), (3, 0), (2, 2), (4, 0)]:
        _run(gpu_lib, x, y, 32, 256, 0, 0, xoff=xo, yoff=yo)
        _run(gpu_lib, x, y, 32, 256, 0, 64, xoff=xo, yoff=yo)
        _run(gpu_lib, x, y, 5, 128, 0, 1024, xoff=xo, yoff=yo)


@pytest.fixture(scope="module")
def axpy_inputs():
    n = 1 << 26
    x, y = synth.f32_normal(n, synth.SEED_AXPY_X), synth.f32_normal(n, synth.SEED_AXPY_Y)
    return x, y, oracle.axpy_sum(A, x, y, 0.0)


@pytest.mark.parametrize("chunk", [0, 1, 64, 1024])
@pytest.mark.parametrize("teams", [64, 128, 256, 512, 1024, 2048, 4096])
def test_axpy_2pow26(gpu_lib, axpy_inputs, chunk, teams):
    x, y, ref = axpy_inputs
    _run(gpu_lib, x, y, teams, 256, 0, chunk, ref=ref)


@pytest.mark.parametrize("chunk", [0, 1, 64, 1024])
def test_axpy_2pow26_default_launch(gpu_lib, axpy_inputs, chunk):
    """The runtime's own choice of teams and threads (the configuration it times)."""
    x, y, ref = axpy_inputs
    _run(gpu_lib, x, y, 0, 0, 0, chunk, ref=ref)
