"""GPU parity of the generic-mode region (power iteration on a diagonal
matrix; teams whose main thread runs the sequential code) against the
oracle's FP64 power iteration on the same fp32 inputs, with one team and
with co-resident teams sharing the sum through an all-gather.

Tolerance, from the arithmetic: the kernel rounds each product, square and
the normalisation in fp32 (unit roundoff u = 2^-24), the oracle does not.
Each step adds a few u of relative error to every component and
normalisation removes the common part, so the spread grows at most
linearly: per component and for lambda, |got - ref| <= 8 (iters + 2) u |ref|.
The start data keep every component far above fp32 underflow.

Cases: ragged sizes across the loop's unroll tile (8 x threads elements),
every team size the entry point takes at both ends, 1 to 64 steps; 2 to 512
teams, also more teams than elements (empty team blocks); launches back to
back with changing team counts and plain reductions in between on the same
stream (the all-gather's tags must stay fresh), with a clean workspace
status; closed forms that come out exact in fp32 (unit vectors, one
element); the zero vector (NaN / infinity propagate identically); the timed
workload sizes.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def run(om, d, v0, iters, teams=1, threads=0):
    dd = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda()
    vv = torch.from_numpy(np.array(v0, dtype=np.float32)).cuda()
    lam = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    om.generic_power(dd, vv, iters, lam, teams=teams, threads=threads)
    torch.cuda.synchronize()
    return vv.cpu().numpy(), float(lam.item())


def check(om, d, v0, iters, teams=1, threads=0):
    got_v, got_l = run(om, d, v0, iters, teams, threads)
    ref_v, ref_l = oracle.power_iteration(np.asarray(d, np.float64), np.asarray(v0, np.float64), iters)
    tol = 8 * (iters + 2) * U
    err = np.abs(got_v.astype(np.float64) - ref_v)
    bad = np.nonzero(err > tol * np.abs(ref_v))[0]
    case = (len(d), iters, teams, threads)
    assert bad.size == 0, (case, bad[:5], got_v[bad[:5]], ref_v[bad[:5]])
    assert abs(got_l - ref_l) <= tol * abs(ref_l), (case, got_l, ref_l)
    assert om.workspace_status() == 0, case


@pytest.mark.parametrize("threads", [64, 256, 1024])
def test_ragged_sizes(gpu_lib, threads):
    for k, n in enumerate([1, 2, 63, 64, 65, 1000, 8 * threads - 1, 8 * threads + 1, 65537, 300001]):
        d, v0 = synth.power_inputs(n, 100 + k)
        for iters in (1, 3, 17):
            check(gpu_lib, d, v0, iters, 1, threads)


@pytest.mark.parametrize("teams,threads", [(2, 64), (7, 256), (64, 1024), (256, 512), (512, 1024)])
def test_coresident_teams(gpu_lib, teams, threads):
    for k, n in enumerate([1, 5, teams - 1, teams + 3, 8 * threads * teams + 17, 300001]):
        if n < 1:
            continue
        d, v0 = synth.power_inputs(n, 300 + k)
        for iters in (1, 2, 9):
            check(gpu_lib, d, v0, iters, teams, threads)


def test_default_teams_and_back_to_back(gpu_lib):
    """Launches of changing team counts, the default choice and plain reductions share the
    stream's workspace; each must see fresh tags."""
    d, v0 = synth.power_inputs(200000, 21)
    x = torch.from_numpy(synth.f32_normal(100000, 22)).cuda()
    s = torch.zeros(1, dtype=torch.float32, device="cuda")
    for teams in (0, 3, 0, 256, 1, 40, 0):
        check(gpu_lib, d, v0, 5, teams)
        gpu_lib.reduce(x, "sum", s, config={"teams": 300})
        check(gpu_lib, d, v0, 4, teams)
    torch.cuda.synchronize()
    assert gpu_lib.workspace_status() == 0


def test_many_steps(gpu_lib):
    d, v0 = synth.power_inputs(20000, 7)
    check(gpu_lib, d, v0, 64, 1)
    check(gpu_lib, d, v0, 64, 16)


@pytest.mark.parametrize("teams", [1, 3])
def test_unit_vector_and_single_element_exact(gpu_lib, teams):
    d = np.array([3.0, -7.0, 0.5, 2.0, 1.25], np.float32)
    for j in range(5):
        v0 = np.zeros(5, np.float32)
        v0[j] = 1.0
        v, lam = run(gpu_lib, d, v0, 5, teams)
        assert np.array_equal(np.abs(v), v0) and lam == abs(d[j])
    # n = 1: v0 = 2, d = -3: w = -6, v = -1, lambda 6; then w = 3, v = 1, lambda 3
    v, lam = run(gpu_lib, [-3.0], [2.0], 1, teams)
    assert v[0] == -1.0 and lam == 6.0
    v, lam = run(gpu_lib, [-3.0], [2.0], 2, teams)
    assert v[0] == 1.0 and lam == 3.0


@pytest.mark.parametrize("teams", [1, 5])
def test_zero_vector(gpu_lib, teams):
    d, _ = synth.power_inputs(777, 3)
    z = np.zeros(777, np.float32)
    for iters in (1, 2):
        v, lam = run(gpu_lib, d, z, iters, teams)
        ref_v, ref_l = oracle.power_iteration(d.astype(np.float64), z.astype(np.float64), iters)
        assert np.isnan(v).all() and np.isnan(ref_v).all()
        assert (lam == ref_l == 0.0) if iters == 1 else (np.isnan(lam) and np.isnan(ref_l))


def test_timed_workload_sizes(gpu_lib):
    # the benchmark's cases: 2^12, 2^16 and 2^20 elements, 100 steps, one team and the
    # default teams
    for n in (1 << 12, 1 << 16, 1 << 20):
        d, v0 = synth.power_inputs(n, 11)
        check(gpu_lib, d, v0, 100, 1)
        check(gpu_lib, d, v0, 100, 0)
