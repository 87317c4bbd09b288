"""Autotuner and timing database for the learned launch-configuration picker.

For each instance (n, dtype, op, body, user chunk) every class of a fixed
candidate grid is timed on the GPU through the library (HIP events on the
launch stream, minimum over repetitions), plus the runtime's built-in
heuristic.  Records go to an append-only JSONL file keyed by instance id,
so an interrupted run resumes where it stopped.  The autotuner's choice for
an instance is the argmin class; it labels the network's training data and
judges its regret.

Class grid (32 classes, shared with the model file's class table):
threads {128, 256, 512, 1024} x teams per CU {1, 2, 4, 8} x unroll {2, 4},
16-byte loads.  Teams for a call = min(teams_per_cu * CUs,
ceil(n * bytes_per_iter / (threads * 16))), at least 1 -- the same rule the
runtime applies when the model picks a class.  For the AXPY body only teams
and threads matter, so unroll-2 and unroll-4 classes of the same
(teams, threads) share one timing.

    python -m paper_2106_03219_amd.tune --out DB.jsonl --count 20000 --seed 7
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

THREADS = (128, 256, 512, 1024)
TEAMS_PER_CU = (1, 2, 4, 8)
UNROLLS = (2, 4)
VEC = 16
CLASSES = [(tpc, th, VEC, un) for th in THREADS for tpc in TEAMS_PER_CU for un in UNROLLS]

ELEM_BYTES = {0: 4, 1: 8, 2: 4, 3: 8, 4: 2}
AXPY_A = 0.7


def class_teams(cls, n, bytes_per_iter, cus):
    tpc, threads, vec, _ = cls
    work = -(-(n * bytes_per_iter) // (threads * vec))
    return int(max(1, min(tpc * cus, work, 65535)))


def class_config(cls, n, bytes_per_iter, cus):
    tpc, threads, vec, unroll = cls
    return {"teams": class_teams(cls, n, bytes_per_iter, cus), "threads": threads, "vec": vec,
            "unroll": unroll}


class Buffers:
    """One max-size device buffer per dtype; instances use prefix views."""

    def __init__(self, max_n, seed=1234):
        import synth
        import torch
        self.torch = torch
        self.t = {}
        for dt in (synth.I32, synth.I64, synth.F32, synth.BF16):
            self.t[dt] = synth.device(dt, max_n, seed + dt)
        self.y = synth.device(synth.F32, max_n, seed + 10)
        self.x_out = {dt: torch.zeros(1, dtype=torch.float64, device="cuda") for dt in self.t}

    def x_for(self, dtype, op):
        torch = self.torch
        if dtype == 4 and op == 0:
            return torch.zeros(1, dtype=torch.float32, device="cuda")
        return torch.zeros(1, dtype=self.t[dtype].dtype, device="cuda")


def time_call(fn, reps, torch):
    """Min over reps of single-launch durations (HIP events on the current stream)."""
    fn()   # warm
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return min(a.elapsed_time(b) for a, b in evs) * 1e3   # microseconds


def tune_instance(om, bufs, inst, cus, torch):
    n, dt, op, body, chunk = inst["n"], inst["dtype"], inst["op"], inst["body"], inst["chunk"]
    bpi = 12 if body else ELEM_BYTES[dt]
    big = n * bpi > (64 << 20)
    reps = 3 if big else 5
    times = []
    cache = {}
    if body:
        x = bufs.t[2][:n]
        y = bufs.y[:n]
        s = torch.zeros(1, dtype=torch.float32, device="cuda")
        c = 0 if chunk < 0 else chunk
        for cls in CLASSES:
            cfg = class_config(cls, n, bpi, cus)
            key = (cfg["teams"], cfg["threads"])
            if key not in cache:
                cache[key] = time_call(lambda: om.axpy_sum(AXPY_A, x, y, s, cfg["teams"], cfg["threads"],
                                                           0, c), reps, torch)
            times.append(cache[key])
        hcfg, _ = om.resolve_config(n, dt, op, 1, chunk, {"flags": om.CFG_NO_MODEL})
        t_heur = time_call(lambda: om.axpy_sum(AXPY_A, x, y, s, 0, 0, 0, c,
                                               config={"flags": om.CFG_NO_MODEL}), reps, torch)
    else:
        inp = bufs.t[dt][:n]
        xo = bufs.x_for(dt, op)
        cfgs = {}
        for cls in CLASSES:
            cfg = class_config(cls, n, bpi, cus)
            key = tuple(cfg.values())
            if key not in cache:
                cache[key] = time_call(lambda: om.reduce(inp, op, xo, config=cfg), reps, torch)
                cfgs[key] = cfg
            times.append(cache[key])
        hcfg, _ = om.resolve_config(n, dt, op, 0, -1, {"flags": om.CFG_NO_MODEL})
        t_heur = time_call(lambda: om.reduce(inp, op, xo, config=hcfg), reps, torch)
        check_consistent(om, inp, dt, op, list(cfgs.values()) + [hcfg], torch)
    return times, t_heur


def check_consistent(om, inp, dt, op, cfgs, torch):
    """Every timed configuration must produce the same reduction from the identity:
    bit-identical for integers and max/min, within 2e-6 relative for compensated
    floating sums (each is within 1e-6 of the exact sum).  Raises otherwise."""
    one = [bufs_identity(torch, dt, op) for _ in cfgs]
    for cfg, x in zip(cfgs, one):
        om.reduce(inp, op, x, config=cfg)
    torch.cuda.synchronize()
    vals = [float(x.float().item()) if x.dtype == torch.bfloat16 else x.item() for x in one]
    if op == 0 and dt in (2, 3, 4):
        ref = max(abs(v) for v in vals)
        if ref > 0 and (max(vals) - min(vals)) > 2e-6 * ref:
            raise RuntimeError(f"configurations disagree on a floating sum: {vals}")
    elif len(set(vals)) != 1:
        raise RuntimeError(f"configurations disagree: {vals}")


def bufs_identity(torch, dt, op):
    tdt = {0: torch.int32, 1: torch.int64, 2: torch.float32, 3: torch.float64,
           4: torch.bfloat16}[dt]
    if dt == 4 and op == 0:
        tdt = torch.float32
    if op == 0:
        return torch.zeros(1, dtype=tdt, device="cuda")
    if dt in (0, 1):
        info = torch.iinfo(tdt)
        return torch.full((1,), info.min if op == 1 else info.max, dtype=tdt, device="cuda")
    return torch.full((1,), -float("inf") if op == 1 else float("inf"), dtype=tdt, device="cuda")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--max-n", type=float, default=1e9)
    ap.add_argument("--limit-s", type=float, default=0, help="stop after this many seconds (resume later)")
    args = ap.parse_args(argv)

    import torch

    import paper_2106_03219_amd as om
    import synth
    om.load()
    om.model_load(None)
    inst = synth.cost_instances(args.count, args.seed)
    inst["n"] = inst["n"].clip(max=int(args.max_n))
    done = set()
    if os.path.exists(args.out):
        for line in open(args.out):
            try:
                done.add(json.loads(line)["id"])
            except (ValueError, KeyError):
                pass
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    max_n = int(inst["n"].max())
    bufs = Buffers(max_n)
    t0 = time.time()
    todo = [i for i in range(args.count) if i not in done]
    print(f"[tune] {len(done)} done, {len(todo)} to go, max n {max_n}, {cus} CUs", flush=True)
    with open(args.out, "a") as fh:
        for k, i in enumerate(todo):
            rec = {"id": i, "n": int(inst["n"][i]), "dtype": int(inst["dtype"][i]),
                   "op": int(inst["op"][i]), "body": int(inst["body"][i]),
                   "chunk": int(inst["chunk"][i])}
            times, th = tune_instance(om, bufs, rec, cus, torch)
            rec["times_us"] = [round(t, 3) for t in times]
            rec["heuristic_us"] = round(th, 3)
            fh.write(json.dumps(rec) + "\n")
            if k % 500 == 0:
                fh.flush()
                print(f"[tune] {k}/{len(todo)} instances, {time.time() - t0:.0f} s", flush=True)
            if args.limit_s and time.time() - t0 > args.limit_s:
                print(f"[tune] time limit reached after {k + 1} instances", flush=True)
                break
    print(f"[tune] finished in {time.time() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
