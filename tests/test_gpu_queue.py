"""GPU parity of dynamic / guided worksharing against the oracle's queues.

The owner of a chunk is not defined for these schedules, so the map check is:
every iteration runs exactly once; the chunk each iteration ran in (its first
iteration, recorded by the kernel) is exactly the oracle's chunk; all
iterations of a chunk ran on one thread; that thread belongs to the team
whose distribute block holds the chunk.  The AXPY body must give y bit for
bit and the sum within 1e-6 of the FP64 oracle, for both kinds and several
chunk sizes, including the 2^26 workload.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check_axpy

pytestmark = pytest.mark.gpu

SCHEDS = [(1, 1, 64, 0, 0, 1), (100, 1, 4, 0, 1, 1), (1000, 3, 96, 0, 0, 1), (100003, 13, 96, 0, 7, 1),
          (100003, 13, 96, 1000, 3, 2), (1 << 20, 64, 256, 0, 1, 1), (1 << 20, 64, 256, 0, 1, 4),
          (1 << 20, 64, 256, 0, 64, 1), (70000, 4096, 64, 0, 0, 1), (12345, 5, 1024, 777, 0, 3),
          (5000, 2, 130, 0, 2, 1)]


def oracle_chunks(kind, n, T, P, dc, c):
    start = np.full(n, -1, dtype=np.int64)
    team = np.full(n, -1, dtype=np.int64)
    chunks = []
    for k in range(T):
        for lo, hi in oracle.team_queue(kind, n, T, P, dc, c, k):
            start[lo:hi] = lo
            team[lo:hi] = k
            chunks.append((lo, hi))
    return start, team, chunks


@pytest.mark.parametrize("kind", ["dynamic", "guided"])
@pytest.mark.parametrize("sched", range(len(SCHEDS)))
def test_queue_map(gpu_lib, kind, sched):
    om = gpu_lib
    n, T, P, dc, c, tickets = SCHEDS[sched]
    owner = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    count = torch.zeros(n, dtype=torch.int32, device="cuda")
    start = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    om.queue_map(kind, n, T, P, dc, c, owner, count, start, tickets=tickets)
    torch.cuda.synchronize()
    owner, count, start = owner.cpu().numpy(), count.cpu().numpy(), start.cpu().numpy()
    ref_start, ref_team, chunks = oracle_chunks(kind, n, T, P, dc, c)
    assert np.all(count == 1)
    assert np.array_equal(start, ref_start)
    assert np.array_equal(owner // P, ref_team)
    assert np.all(owner % P < P) and np.all(owner >= 0)
    for lo, hi in chunks:
        assert np.all(owner[lo:hi] == owner[lo]), (lo, hi)


AXPY = [(1000, 3, 96, 0, 0), (100003, 13, 96, 0, 1), (100003, 13, 96, 1000, 3), (1 << 20, 64, 256, 0, 64),
        (1 << 20, 0, 0, 0, 1), (1 << 20, 0, 0, 0, 0), (5000, 2, 130, 0, 2),
        # whole-wave teams with long chunks (through LDS lines): ragged chunk
        # sizes and block starts, distribute blocks, a final partial round
        ((1 << 20) + 37, 5, 192, 0, 100), (300000, 7, 512, 30011, 64), ((1 << 20) + 3, 3, 128, 0, 2048),
        # short dynamic chunks as the union of a wave's runs: on and off the
        # line grid, a final partial round, the runtime's own team size
        ((1 << 20) + 37, 5, 192, 0, 16), ((1 << 20), 4, 256, 0, 32), (300001, 7, 256, 0, 48),
        ((1 << 20) + 11, 0, 0, 0, 64), (200003, 3, 64, 0, 24), ((1 << 20), 8, 512, 0, 64),
        # short dynamic chunks off the line grid (8 to 15: the union of a wave's runs;
        # 7 and 4: lane by lane)
        ((1 << 20) + 37, 5, 192, 0, 8), (300001, 7, 256, 0, 12), (200003, 3, 64, 0, 15),
        (300001, 0, 0, 0, 8), ((1 << 20) + 37, 5, 192, 0, 7), (300001, 7, 256, 0, 4),
        # dynamic chunks of 16 and 17 lines (a wave's lines in a rotated order)
        ((1 << 21) + 37, 5, 192, 0, 544), (37 * 64 * 1024, 37, 64, 0, 512)]


@pytest.mark.parametrize("kind", ["dynamic", "guided"])
@pytest.mark.parametrize("case", range(len(AXPY)))
def test_queue_axpy_parity(gpu_lib, kind, case):
    om = gpu_lib
    n, T, P, dc, c = AXPY[case]
    xh = synth.f32_normal(n, 4)
    yh = synth.f32_normal(n, 5)
    ref_y, ref_s = oracle.axpy_sum(0.7, xh, yh, 0.25)
    x, y = torch.from_numpy(xh).cuda(), torch.from_numpy(yh.copy()).cuda()
    s = torch.tensor([0.25], dtype=torch.float32, device="cuda")
    om.axpy_sum_queue(kind, 0.7, x, y, s, T, P, dc, c)
    torch.cuda.synchronize()
    check_axpy(y.cpu().numpy(), s.item(), ref_y, ref_s, 0.25, (kind, AXPY[case]))


def test_queue_axpy_2pow26_all_chunks_agree(gpu_lib):
    om = gpu_lib
    n = 1 << 26
    x = synth.device(synth.F32, n, synth.SEED_AXPY_X)
    y0 = synth.device(synth.F32, n, synth.SEED_AXPY_Y)
    ys = []
    for kind, c in (("dynamic", 1), ("dynamic", 64), ("dynamic", 1024), ("guided", 1), ("guided", 64)):
        y = y0.clone()
        s = torch.zeros(1, dtype=torch.float32, device="cuda")
        om.axpy_sum_queue(kind, 0.7, x, y, s, chunk=c)
        torch.cuda.synchronize()
        ys.append((y, float(s.item())))
    yref = y0.clone()
    sref = torch.zeros(1, dtype=torch.float32, device="cuda")
    om.axpy_sum(0.7, x, yref, sref)          # the static schedule
    torch.cuda.synchronize()
    for y, sv in ys:
        assert torch.equal(y, yref)
        assert abs(sv - float(sref.item())) <= 1e-6 * abs(float(sref.item()))
    # sampled elements against the oracle's single rounding
    idx = np.random.Generator(np.random.PCG64(9)).integers(0, n, 4096)
    xh, yh = x[idx].cpu().numpy(), y0[idx].cpu().numpy()
    ry, _ = oracle.axpy_sum(0.7, xh, yh)
    assert np.array_equal(yref[idx].cpu().numpy().view(np.uint32), ry.view(np.uint32))
