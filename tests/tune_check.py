"""Oracle check of the autotuner's timed runs.

Every record of a timing database (paper_2106_03219_amd.tune) keeps the
result each distinct configuration computed.  The instances are prefixes of
a few shared device buffers drawn from fixed seeds, so the check redraws
those buffers, copies them to the host, and lets the oracle fold each
(dtype, op) group once at every prefix length the group uses
(oracle.fold_prefixes; AXPY sums: oracle.axpy_prefix_sums).  Integer sums
and every max / min must match bit for bit; floating sums within 1e-6 of
the FP64 value.  Needs the GPU only to redraw the buffers.

    python tests/tune_check.py DB.jsonl [DB2.jsonl ...]
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OPN = {0: "sum", 1: "max", 2: "min"}
TOL = 1e-6


def host_buffers(buffer_n: int):
    """Host copies of the tuner's shared buffers of length buffer_n (drawn on the GPU
    with the tuner's seeds): {dtype: array} (bf16 as uint16 bits) and y0."""
    import torch

    from paper_2106_03219_amd.tune import BUFFER_SEED
    out = {}
    for dt in (synth.I32, synth.I64, synth.F32, synth.BF16):
        t = synth.device(dt, buffer_n, BUFFER_SEED + dt)
        out[dt] = (t.view(torch.int16).cpu().numpy().view(np.uint16) if dt == synth.BF16
                   else t.cpu().numpy())
        del t
    y0 = synth.device(synth.F32, buffer_n, BUFFER_SEED + 10).cpu().numpy()
    return out, y0


def _close(got, ref, dt, op):
    if dt in (synth.I32, synth.I64) or op != 0:
        return (int(got) == int(ref)) if dt in (synth.I32, synth.I64) else (float(got) == float(ref))
    if ref == 0.0:
        return abs(float(got)) <= TOL
    return abs(float(got) - ref) <= TOL * abs(ref)


def check_records(recs, log=print):
    """Check every recorded result against the oracle.  Returns a summary dict;
    raises AssertionError listing the first mismatches."""
    from paper_2106_03219_amd.tune import AXPY_A
    by_buf = {}
    for r in recs:
        by_buf.setdefault(int(r["buffer_n"]), []).append(r)
    checked, worst_rel, bad = 0, 0.0, []
    for buffer_n, rs in sorted(by_buf.items()):
        host, y0 = host_buffers(buffer_n)
        groups = {}
        for r in rs:
            key = ("axpy",) if r["body"] else (int(r["dtype"]), int(r["op"]))
            groups.setdefault(key, []).append(r)
        for key, grp in groups.items():
            lens = [int(r["n"]) for r in grp]
            if key == ("axpy",):
                _, refs = oracle.axpy_prefix_sums(AXPY_A, host[synth.F32], y0, lens)
                dt, op = synth.F32, 0
            else:
                dt, op = key
                refs = oracle.fold_prefixes(host[dt], OPN[op], lens, bf16=dt == synth.BF16)
            for r, ref in zip(grp, refs):
                for res in r["results"]:
                    got = res[4]
                    checked += 1
                    if dt not in (synth.I32, synth.I64) and op == 0 and ref != 0.0:
                        worst_rel = max(worst_rel, abs(float(got) - ref) / abs(ref))
                    if not _close(got, ref, dt, op):
                        bad.append((r["id"], key, r["n"], res, ref))
        del host, y0
    summary = {"records": len(recs), "results_checked": checked,
               "worst_rel_fp_sum": worst_rel, "mismatches": len(bad)}
    log(f"[tune_check] {summary}")
    assert not bad, bad[:10]
    return summary


def main(argv):
    recs = []
    for path in argv:
        recs += [json.loads(line) for line in open(path) if line.strip()]
    check_records(recs)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
