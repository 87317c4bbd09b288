"""Autotuner and timing database for the learned launch-configuration picker.

For each instance (n, dtype, op, body, user chunk) every class of a fixed
candidate grid is timed on the GPU through the library (HIP events on the
launch stream, minimum over repetitions), plus the runtime's built-in
heuristic.  The time of a class is the GPU time a launch adds to a stream of
launches: a batch of launches is queued behind a spin kernel and timed as a
whole, so host enqueueing leaves no gaps.  Each timed launch reads a window
of the shared buffers that no launch has touched since the buffers were last
traversed, so it streams from HBM as a reduction over resident data does
(repeating one small input would time the 256 MB Infinity Cache instead).  Records go to an append-only JSONL file keyed by instance id,
so an interrupted run resumes where it stopped.  The autotuner's choice for
an instance is the argmin class; it labels the network's training data and
judges its regret.

Class grid (64 classes, shared with the model file's class table):
threads {128, 256, 512, 1024} x teams per CU {1, 2, 4, 8} x bytes per lane
per load {8, 16} x loads in flight {2, 4}.  Teams for a call =
min(teams_per_cu * CUs, ceil(n * bytes_per_iter / (threads * vec))), at
least 1 -- the same rule the runtime applies when the model picks a class.
For the AXPY body only teams and threads matter (its kernel fixes its own
loads), so classes that give the same (teams, threads) share one timing.

Every record also keeps the result each distinct configuration computed
(plain reductions from the op's identity; AXPY sums from a pristine y and a
zero sum), so the timed runs can be checked against an independent
reference afterwards: the instances are prefixes of a few shared buffers,
whose host copies a checker folds once per (dtype, op) at every prefix
length.

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
VECS = (8, 16)
UNROLLS = (2, 4)
CLASSES = [(tpc, th, vec, un) for th in THREADS for tpc in TEAMS_PER_CU for vec in VECS
           for un in UNROLLS]

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


BUFFER_SEED = 1234


class Buffers:
    """One max-size device buffer per dtype (seed BUFFER_SEED + dtype code) and the
    AXPY y (seed BUFFER_SEED + 10, kept pristine in y0); instances use prefix views."""

    def __init__(self, max_n, seed=BUFFER_SEED):
        import synth
        import torch
        self.torch = torch
        self.t = {}
        for dt in (synth.I32, synth.I64, synth.F32, synth.BF16):
            self.t[dt] = synth.device(dt, max_n, seed + dt)
        self.y0 = synth.device(synth.F32, max_n, seed + 10)
        self.y = self.y0.clone()
        self.n = max_n
        self.cursor = [0]   # next timing window (shared by every instance)

    def x_for(self, dtype, op):
        torch = self.torch
        if dtype == 4 and op == 0:
            return torch.zeros(1, dtype=torch.float32, device="cuda")
        return torch.zeros(1, dtype=self.t[dtype].dtype, device="cuda")


def time_call(fn, reps, torch, windows=None):
    """GPU time per launch of fn, min over reps (HIP events on the current stream).

    Without `windows`: single launches, one event pair each.  With `windows` (a Windows of
    the instance's length): the GPU time a launch adds to a stream of launches.  Each rep
    enqueues a spin kernel long enough to cover the host's enqueueing, then an event, then
    `windows.k` launches of fn back to back, then an event: the launches run from the queue
    without host gaps, and the time per launch is the span over k.  Every launch reads a
    window of the shared buffers that no launch has touched since the buffers were last
    traversed, so it streams its input from HBM as a reduction over resident data does
    (repeating one small input would time the 256 MB Infinity Cache instead).  fn then takes
    the window's element offset."""
    if windows is None:
        fn()   # warm
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return min(a.elapsed_time(b) for a, b in evs) * 1e3   # microseconds
    fn(windows.next())   # warm (code, configuration caches)
    best = float("inf")
    for _ in range(reps):
        offs = [windows.next() for _ in range(windows.k)]
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(SPIN_CYCLES[0])
        a.record()
        for o in offs:
            fn(o)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) * 1e3 / len(offs))
    return best


# Spin-kernel cycles that keep the GPU busy for about 150 µs, enough to cover the host
# enqueueing a batch of timed launches (set by calibrate_spin).
SPIN_CYCLES = [1 << 20]


def calibrate_spin(torch, target_us=150.0):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(1 << 20)
    a.record()
    torch.cuda._sleep(1 << 20)
    b.record()
    torch.cuda.synchronize()
    us = max(a.elapsed_time(b) * 1e3, 1.0)
    SPIN_CYCLES[0] = int((1 << 20) * target_us / us)
    return us


class Windows:
    """Element offsets of successive windows of n elements in buffers of buffer_n elements:
    a cursor that moves on by n (rounded up to 64 elements, 256 B of 4-byte data) per window
    and wraps round at the end, so a window is read again only after the whole buffer.  k:
    launches timed back to back (8, or 3 for inputs above 64 MiB)."""

    def __init__(self, cursor, n, buffer_n, k=8):
        self.c, self.n, self.buffer_n, self.k = cursor, n, buffer_n, k

    def next(self):
        step = (self.n + 63) // 64 * 64
        if self.c[0] + self.n > self.buffer_n:
            self.c[0] = 0
        o = self.c[0]
        self.c[0] += step
        return o


def _value(x):
    return float(x.float().item()) if x.dtype.is_floating_point else int(x.item())


def tune_instance(om, bufs, inst, cus, torch):
    """Times of every class (in CLASSES order) and of the heuristic for one instance,
    and the distinct configurations' results: a list of [teams, threads, vec, unroll,
    value] (AXPY: [teams, threads, 0, 0, sum]); the heuristic's is the last."""
    n, dt, op, body, chunk = inst["n"], inst["dtype"], inst["op"], inst["body"], inst["chunk"]
    bpi = 12 if body else ELEM_BYTES[dt]
    big = n * bpi > (64 << 20)
    reps = 2
    times = []
    cache = {}
    results = []
    if body:
        x = bufs.t[2][:n]
        y = bufs.y[:n]
        s = torch.zeros(1, dtype=torch.float32, device="cuda")
        c = 0 if chunk < 0 else chunk

        def axpy(teams, threads, config=None):
            return lambda: om.axpy_sum(AXPY_A, x, y, s, teams, threads, 0, c, config=config)

        def axpy_at(teams, threads, config=None):   # timed launches, on rotating windows
            return lambda o: om.axpy_sum(AXPY_A, bufs.t[2][o:o + n], bufs.y[o:o + n], s, teams,
                                         threads, 0, c, config=config)
        win = Windows(bufs.cursor, n, bufs.n, 3 if big else 8)

        def result(run):
            y.copy_(bufs.y0[:n])
            s.zero_()
            run()
            return _value(s)
        for cls in CLASSES:
            cfg = class_config(cls, n, bpi, cus)
            key = (cfg["teams"], cfg["threads"])
            if key not in cache:
                cache[key] = time_call(axpy_at(*key), reps, torch, win)
                results.append([key[0], key[1], 0, 0, result(axpy(*key))])
            times.append(cache[key])
        heur = axpy(0, 0, {"flags": om.CFG_NO_MODEL})
        t_heur = time_call(axpy_at(0, 0, {"flags": om.CFG_NO_MODEL}), reps, torch, win)
        results.append([0, 0, 0, 0, result(heur)])
        y.copy_(bufs.y0[:n])
    else:
        inp = bufs.t[dt][:n]
        full = bufs.t[dt]
        xo = bufs.x_for(dt, op)
        win = Windows(bufs.cursor, n, bufs.n, 3 if big else 8)
        cfgs = []
        for cls in CLASSES:
            cfg = class_config(cls, n, bpi, cus)
            key = tuple(cfg.values())
            if key not in cache:
                cache[key] = time_call(lambda o: om.reduce(full[o:o + n], op, xo, config=cfg),
                                       reps, torch, win)
                cfgs.append(cfg)
            times.append(cache[key])
        hcfg, _ = om.resolve_config(n, dt, op, 0, -1, {"flags": om.CFG_NO_MODEL})
        t_heur = time_call(lambda o: om.reduce(full[o:o + n], op, xo, config=hcfg), reps, torch,
                           win)
        cfgs.append(hcfg)
        outs = [bufs_identity(torch, dt, op) for _ in cfgs]
        for cfg, xv in zip(cfgs, outs):
            om.reduce(inp, op, xv, config=cfg)
        torch.cuda.synchronize()
        results = [[cfg["teams"], cfg["threads"], cfg["vec"], cfg["unroll"], _value(xv)]
                   for cfg, xv in zip(cfgs, outs)]
    return times, t_heur, results


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
    spin = calibrate_spin(torch)
    bufs = Buffers(max_n)
    t0 = time.time()
    todo = [i for i in range(args.count) if i not in done]
    print(f"[tune] {len(done)} done, {len(todo)} to go, max n {max_n}, {cus} CUs, spin 2^20 "
          f"cycles {spin:.0f} us", flush=True)
    with open(args.out, "a") as fh:
        for k, i in enumerate(todo):
            rec = {"id": i, "n": int(inst["n"][i]), "dtype": int(inst["dtype"][i]),
                   "op": int(inst["op"][i]), "body": int(inst["body"][i]),
                   "chunk": int(inst["chunk"][i])}
            times, th, results = tune_instance(om, bufs, rec, cus, torch)
            rec["times_us"] = [round(t, 3) for t in times]
            rec["heuristic_us"] = round(th, 3)
            rec["results"] = results
            rec["buffer_n"] = max_n
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
