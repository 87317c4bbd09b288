"""The autotuner end to end on a handful of instances: every class of the
grid (threads x teams per CU x vector width x loads in flight) is timed, the
records are well formed, and every distinct configuration's result is
checked against the oracle (tests/tune_check.py).
"""
import json

import pytest
import torch

import synth
import tune_check

pytestmark = pytest.mark.gpu


def test_tuner_records_match_oracle(gpu_lib, tmp_path):
    from paper_2106_03219_amd import tune
    om = gpu_lib
    assert len(tune.CLASSES) == 64
    assert {c[2] for c in tune.CLASSES} == {8, 16}
    db = tmp_path / "db.jsonl"
    # 12 instances of the training distribution, n capped at 2e6 to keep it short
    assert tune.main(["--out", str(db), "--count", "12", "--seed", "77", "--max-n", "2e6"]) == 0
    recs = [json.loads(line) for line in open(db)]
    assert sorted(r["id"] for r in recs) == list(range(12))
    inst = synth.cost_instances(12, 77)
    for r in recs:
        assert r["n"] == min(int(inst["n"][r["id"]]), 2_000_000)
        assert len(r["times_us"]) == 64 and all(t > 0 for t in r["times_us"])
        assert r["heuristic_us"] > 0
        assert r["results"] and r["buffer_n"] >= r["n"]
    summary = tune_check.check_records(recs)
    assert summary["mismatches"] == 0 and summary["results_checked"] >= 12
    # a resumed run adds nothing
    assert tune.main(["--out", str(db), "--count", "12", "--seed", "77", "--max-n", "2e6"]) == 0
    assert len(open(db).read().splitlines()) == 12
    torch.cuda.synchronize()
