"""GPU parity of the histogram reduction (reduction(+: hist[0:bins]) with
hist[key[i]] += 1) against the oracle, exact: bin counts from 1 to 9 000 000
(team copies in LDS -- up to 40 704 bins with gfx950's 160 KiB a workgroup;
two ranges of bins, each in LDS; then the keys partitioned by range of 32 768
bins and each range counted in LDS -- up to 4 194 304 bins every tile of keys
sorted by range into a slot of its own, up to 8 388 608 the ranges laid out
across teams; beyond, atomics on hist itself; on request ranges up to 32 of
them, either partition for any bin count it takes, team copies in the global
pool, or atomics on hist for any bin count), uniform, skewed and single-key
(fully contended) inputs, an incoming histogram taking part, keys out of
range (skipped and flagged), several launch configurations and team counts,
and repeated launches."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

BINS = [1, 7, 256, 4096, 16256, 16257, 40704, 40705, 81408, 81409, 162816, 162817, 520193,
        1 << 20, 1302528, 1302529, 8388608, 8388609]
SIZES = [1, 1000, (1 << 20) | 5]


def run(om, keys, bins, hist0, config=None):
    k = torch.from_numpy(np.ascontiguousarray(keys, dtype=np.int32)).cuda()
    h = torch.from_numpy(np.array(hist0, dtype=np.int32)).cuda()
    om.histogram(k, bins, h, config=config)
    torch.cuda.synchronize()
    return h.cpu().numpy()


@pytest.mark.parametrize("bins", BINS)
def test_uniform_keys(gpu_lib, bins):
    g = np.random.Generator(np.random.PCG64(bins))
    for n in SIZES:
        keys = g.integers(0, bins, n).astype(np.int32)
        h0 = g.integers(-1000, 1000, bins).astype(np.int32)
        want, sk = oracle.histogram(keys, bins, hist=h0)
        assert sk == 0
        assert np.array_equal(run(gpu_lib, keys, bins, h0), want)


@pytest.mark.parametrize("flag", ["HIST_TEAM_COPY", "HIST_DIRECT", "HIST_PARTITION", "HIST_RANGES",
                                  "HIST_TILE_SORT"])
@pytest.mark.parametrize("bins", [7, 16257, 32769, 1 << 20, 1400000, 2097153, 4194304, 4194305])
def test_forced_strategies(gpu_lib, flag, bins):
    """Team copies from the global pool (team-shared allocation falling back past LDS) and
    atomics on hist, each forced where the default would choose otherwise (the pool holds a
    full copy per team: 16 teams keep it small)."""
    g = np.random.Generator(np.random.PCG64(bins + 11))
    cfg = {"flags": getattr(gpu_lib, "CFG_" + flag)}
    if flag == "HIST_TEAM_COPY":
        cfg["teams"] = 16
    if flag == "HIST_TILE_SORT" and bins > 128 * 32768:   # 128 ranges at most: refused
        with pytest.raises(gpu_lib.OmprtError):
            run(gpu_lib, np.zeros(10, dtype=np.int32), bins, np.zeros(bins), cfg)
        return
    for n in (1, 1000, 300001):
        keys = g.integers(0, bins, n).astype(np.int32)
        h0 = g.integers(-1000, 1000, bins).astype(np.int32)
        want, _ = oracle.histogram(keys, bins, hist=h0)
        assert np.array_equal(run(gpu_lib, keys, bins, h0, cfg), want), (flag, bins, n)
    same = np.full(100003, bins // 2, dtype=np.int32)      # every key on one bin
    want, _ = oracle.histogram(same, bins)
    assert np.array_equal(run(gpu_lib, same, bins, np.zeros(bins), cfg), want)


@pytest.mark.parametrize("cfg", [{"teams": 1}, {"teams": 4096, "threads": 64}, {"unroll": 1},
                                 {"threads": 1024, "unroll": 2}])
def test_configs_and_contention(gpu_lib, cfg):
    g = np.random.Generator(np.random.PCG64(5))
    for bins in (300, 50000):
        keys = g.integers(0, bins, 300001).astype(np.int32)
        want, _ = oracle.histogram(keys, bins)
        assert np.array_equal(run(gpu_lib, keys, bins, np.zeros(bins), cfg), want)
        same = np.full(200003, bins - 1, dtype=np.int32)      # every key on one bin
        want, _ = oracle.histogram(same, bins)
        assert np.array_equal(run(gpu_lib, same, bins, np.zeros(bins), cfg), want)


def test_out_of_range_keys_flagged(gpu_lib):
    om = gpu_lib
    g = np.random.Generator(np.random.PCG64(6))
    keys = g.integers(-5, 105, 100000).astype(np.int32)
    want, sk = oracle.histogram(keys, 100)
    assert sk > 0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        om.workspace_reset()
        k = torch.from_numpy(keys).cuda()
        h = torch.zeros(100, dtype=torch.int32, device="cuda")
        om.histogram(k, 100, h)
    s.synchronize()
    assert np.array_equal(h.cpu().numpy(), want)
    assert om.workspace_status(stream=s) & 4
    with torch.cuda.stream(s):
        om.workspace_reset()
    assert om.workspace_status(stream=s) == 0
    # the atomic and the partitioned strategies flag them the same way
    for flag in (om.CFG_HIST_DIRECT, om.CFG_HIST_PARTITION, om.CFG_HIST_TILE_SORT):
        with torch.cuda.stream(s):
            h.zero_()
            om.histogram(k, 100, h, config={"flags": flag})
        s.synchronize()
        assert np.array_equal(h.cpu().numpy(), want)
        assert om.workspace_status(stream=s) & 4
        with torch.cuda.stream(s):
            om.workspace_reset()
    # partitioned by default: keys outside [0, 500000) among valid ones
    big = g.integers(-50, 500050, 400001).astype(np.int32)
    want, sk = oracle.histogram(big, 500000)
    assert sk > 0
    with torch.cuda.stream(s):
        kb = torch.from_numpy(big).cuda()
        hb = torch.zeros(500000, dtype=torch.int32, device="cuda")
        om.histogram(kb, 500000, hb)
    s.synchronize()
    assert np.array_equal(hb.cpu().numpy(), want)
    assert om.workspace_status(stream=s) & 4
    with torch.cuda.stream(s):
        om.workspace_reset()


def test_repeated_launches_accumulate(gpu_lib):
    om = gpu_lib
    g = np.random.Generator(np.random.PCG64(7))
    for bins in (1000, 30000, 200000):
        keys = g.integers(0, bins, 123457).astype(np.int32)
        k = torch.from_numpy(keys).cuda()
        h = torch.zeros(bins, dtype=torch.int32, device="cuda")
        for _ in range(50):
            om.histogram(k, bins, h)
        torch.cuda.synchronize()
        want, _ = oracle.histogram(keys, bins)
        assert np.array_equal(h.cpu().numpy(), 50 * want)


@pytest.mark.parametrize("bins,skew", [(1 << 20, False), (1 << 20, True), (5_000_000, True),
                                       (8388608, False)])
def test_partition_at_scale(gpu_lib, bins, skew):
    """The partitioned strategy (the default from five LDS ranges to 8 388 608 bins) over
    2^26 keys -- many tiles per team, range counts in the millions -- uniform, or skewed so
    that most keys fall into a few ranges (a cubed uniform: the low bins take most), with
    an incoming histogram, exact against the oracle."""
    g = np.random.Generator(np.random.PCG64(bins + int(skew)))
    n = 1 << 26
    if skew:
        keys = (g.random(n) ** 3 * bins).astype(np.int32)
    else:
        keys = g.integers(0, bins, n).astype(np.int32)
    h0 = g.integers(-1000, 1000, bins).astype(np.int32)
    want, sk = oracle.histogram(keys, bins, hist=h0)
    assert sk == 0
    assert np.array_equal(run(gpu_lib, keys, bins, h0), want), (bins, skew)


@pytest.mark.parametrize("flag,teams", [("HIST_PARTITION", t) for t in (1, 7, 100, 1500, 2500)] +
                         [("HIST_TILE_SORT", t) for t in (1, 7, 100, 1500, 2500)])
def test_partition_team_counts(gpu_lib, flag, teams):
    """The forced partitions with team counts that are not whole waves of the per-range scan
    (1, 7, 100), and with more teams than one scan workgroup covers in one piece (1500, 2500:
    the range's counts are scanned 1024 at a time with a carry); for the tile sort (which
    takes no more teams than tiles), teams with several tiles or one partial tile, over 5, 40
    and the most ranges each takes (128, 256)."""
    g = np.random.Generator(np.random.PCG64(teams))
    cfg = {"flags": getattr(gpu_lib, "CFG_" + flag), "teams": teams}
    for bins in (5 * 32768 - 3, 1302529, 4194304 if flag == "HIST_TILE_SORT" else 8388608):
        for n in (1, 4097, 1000003):
            keys = g.integers(0, bins, n).astype(np.int32)
            h0 = g.integers(-1000, 1000, bins).astype(np.int32)
            want, _ = oracle.histogram(keys, bins, hist=h0)
            assert np.array_equal(run(gpu_lib, keys, bins, h0, cfg), want), (teams, bins, n)


def test_tile_sort_team_with_fewer_tiles(gpu_lib):
    """49 153 keys over 3 teams: the first team's block is 16 385 keys (three tiles), the
    others 16 384 (two), so their third tile's run starts are written empty."""
    g = np.random.Generator(np.random.PCG64(31))
    cfg = {"flags": gpu_lib.CFG_HIST_TILE_SORT, "teams": 3}
    for bins in (100000, 2097152, 4194304):
        keys = g.integers(0, bins, 49153).astype(np.int32)
        h0 = g.integers(-1000, 1000, bins).astype(np.int32)
        want, _ = oracle.histogram(keys, bins, hist=h0)
        assert np.array_equal(run(gpu_lib, keys, bins, h0, cfg), want), bins
