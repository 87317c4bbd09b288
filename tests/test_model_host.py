"""Host-side tests of the learned picker (CPU only): the model file the trainer
writes loads into the library, and the library's C++ inference picks the
same class as a numpy forward pass of the same weights; the confidence
threshold falls back to the heuristic; regret / tau bookkeeping of the
trainer on a synthetic timing table.
"""
import numpy as np
import pytest

import paper_2106_03219_amd as om
from paper_2106_03219_amd import train, tune

CUS = 256   # no device here: the library's fallback compute-unit count


def _forward(p, x, dims=train.DIMS):
    F, H1, H2, K = dims
    o = 0
    W1 = p[o:o + H1 * F].reshape(H1, F); o += H1 * F
    b1 = p[o:o + H1]; o += H1
    W2 = p[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = p[o:o + H2]; o += H2
    W3 = p[o:o + K * H2].reshape(K, H2); o += K * H2
    b3 = p[o:o + K]
    h1 = np.maximum(W1.astype(np.float64) @ x + b1, 0)
    h2 = np.maximum(W2.astype(np.float64) @ h1 + b2, 0)
    return W3.astype(np.float64) @ h2 + b3


@pytest.fixture
def model_file(tmp_path):
    g = np.random.Generator(np.random.PCG64(3))
    p = (g.standard_normal(om.mlp_param_count(*train.DIMS)) * 0.5).astype(np.float32)
    mean = g.standard_normal(16).astype(np.float32)
    scale = (0.5 + g.random(16)).astype(np.float32)
    path = tmp_path / "model.txt"
    train.write_model(str(path), mean, scale, p, 0.0)
    yield path, p, mean, scale
    om.model_load(None)


def test_host_inference_matches_numpy_forward(model_file):
    path, p, mean, scale = model_file
    om.model_load(str(path))
    g = np.random.Generator(np.random.PCG64(9))
    checked = 0
    for _ in range(300):
        n = int(10 ** g.uniform(3, 9))
        dt = int(g.choice([om.I32, om.I64, om.F32, om.BF16]))
        op = int(g.integers(0, 3))
        body = int(g.integers(0, 2))
        chunk = int(g.choice([-1, 0, 1, 64, 1024])) if body else -1
        f = np.array(om.model_features(n, dt, op, body, chunk), dtype=np.float32)
        z = _forward(p, ((f - mean) * scale).astype(np.float64))
        s = np.sort(z)
        if s[-1] - s[-2] < 1e-3:        # a near-tie may resolve differently in fp32
            continue
        k = int(np.argmax(z))
        bpi = 12 if body else {0: 4, 1: 8, 2: 4, 4: 2}[dt]
        cfg, src = om.resolve_config(n, dt, op, body, chunk)
        assert src == 1
        assert cfg == tune.class_config(tune.CLASSES[k], n, bpi, CUS)
        checked += 1
    assert checked > 250


def test_threshold_falls_back(tmp_path):
    # all-zero network: uniform softmax (confidence 1/K) below any tau > 1/K
    p = np.zeros(om.mlp_param_count(*train.DIMS), np.float32)
    path = tmp_path / "flat.txt"
    train.write_model(str(path), np.zeros(16, np.float32), np.ones(16, np.float32), p, 0.5)
    om.model_load(str(path))
    try:
        _, src = om.resolve_config(1 << 20, om.F32, "sum")
        assert src == 3
        _, src = om.resolve_config(1 << 20, om.F32, "sum", config={"flags": om.CFG_NO_MODEL})
        assert src == 3
    finally:
        om.model_load(None)


def test_bad_model_files_rejected(tmp_path):
    bad = tmp_path / "bad.txt"
    bad.write_text("omprt-mlp 1\ndims 16 64 64 32\ntau 0\nmean 1 2 3\n")
    with pytest.raises(om.OmprtError):
        om.model_load(str(bad))
    with pytest.raises(om.OmprtError):
        om.model_load(str(tmp_path / "missing.txt"))
    _, src = om.resolve_config(1000, om.F32, "sum")
    assert src == 3      # nothing loaded


def test_regret_and_tau_bookkeeping():
    K = len(tune.CLASSES)
    recs = []
    for i in range(4):
        t = [10.0 + j for j in range(K)]
        recs.append({"times_us": t, "heuristic_us": 20.0})
    pred = np.array([0, 1, 2, 3])
    ev = train.evaluate(recs, pred)
    assert ev["regret_mean"] == pytest.approx(np.mean([0, 0.1, 0.2, 0.3]))
    assert ev["top1_agreement"] == 0.25
    assert ev["gain_vs_heuristic_geomean"] == pytest.approx(np.exp(np.mean(np.log(20 / np.array([10, 11, 12, 13])))))
    conf = np.array([0.9, 0.9, 0.1, 0.1])
    got = train.picked_times(recs, pred, conf, 0.5)
    assert list(got) == [10.0, 11.0, 20.0, 20.0]
    assert train.choose_tau(recs, pred, conf) == 0.0     # the model beats the heuristic everywhere


def test_class_grid_matches_runtime_rule():
    assert len(tune.CLASSES) == 64 and len(set(tune.CLASSES)) == 64
    assert {c[2] for c in tune.CLASSES} == {8, 16} and {c[3] for c in tune.CLASSES} == {2, 4}
    # 8-byte loads need twice the teams of 16-byte ones for the same small input
    assert tune.class_teams((8, 256, 8, 4), 4096, 4, CUS) == 8
    assert tune.class_teams((8, 256, 16, 4), 4096, 4, CUS) == 4
    assert tune.class_teams((8, 256, 16, 4), 10, 4, CUS) == 1
    assert tune.class_teams((8, 256, 16, 4), 1 << 30, 4, CUS) == 8 * CUS
    assert tune.class_teams((1, 1024, 16, 2), 1 << 30, 12, CUS) == CUS


def test_tuner_windows_rotate_inside_the_buffer():
    """The autotuner's timing windows: aligned to 64 elements, inside the buffer, every
    window distinct until the cursor wraps, the cursor shared by all instances."""
    from paper_2106_03219_amd.tune import Windows
    cursor = [0]
    buffer_n = 1_000_000
    seen = []
    for n in (1000, 12345, 64, 999_999, 1):
        w = Windows(cursor, n, buffer_n, k=8)
        for _ in range(50):
            o = w.next()
            assert o % 64 == 0 and 0 <= o and o + n <= buffer_n
            seen.append((o, n))
    firsts = [o for o, n in seen[:50]]
    assert len(set(firsts)) == 50          # no window of the first instance read twice
    assert cursor[0] > 0
    big = Windows(cursor, buffer_n, buffer_n)
    assert {big.next() for _ in range(5)} == {0}   # a window as large as the buffer stays at 0
