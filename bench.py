"""Benchmark of the data-parallel reduction core on one MI355X.

One step = one pass of the plain reduction path over the at-scale
workload: fp32 sum and fp32 max over N = 2^28 elements ~ N(0, 1) and int64
sum over N = 2^28 elements uniform in [-2^40, 2^40] (4 GiB read per step),
inputs resident in HBM, launch configuration chosen by the runtime.  The
printed JSON line reports whole-step throughput in GB/s, the roofline of the
dominant kernel (the int64 sum, timed with HIP events on its stream over
the timed region), and the CPU baseline leg: the oracle timed on the host over
the same step, whose results also check the GPU step.  Unless --no-extras:
the AXPY worksharing body, launch latency, the 4096-segment batched workload
(plain launches vs one graph-replayed persistent launch), device atomics,
array-section reductions, the AXPY body under dynamic / guided schedules,
several reduction variables in one pass, maxloc and histograms, and the
learned picker against the heuristic on held-out instances.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 1 << 28
METRIC = "reduction GB/s (% HBM peak); batched reductions/s learned vs plain at 1e-6"


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "reduce_int64_sum_2pow28_traffic.json")


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    try:
        d = json.load(open(TRAFFIC_FILE))
        h = hashlib.sha256()
        for s in d["sources"]:
            h.update(open(os.path.join(ROOT, s), "rb").read())
        if h.hexdigest()[:16] != d["source_sha256_16"]:
            return None
        return int(d["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(f_host, i_host, passes: int):
    """The CPU baseline leg: the oracle, as is, timed over the same step on one host
    core.  Its results (FP64 Neumaier sum and sum|x|, fmax fold, wrapping int64 sum)
    are also what the GPU step is checked against."""
    import numpy as np
    import oracle
    # pinned to one core of those this process may use (the oracle is serial C)
    allowed = os.sched_getaffinity(0)
    core = min(allowed)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        for _ in range(passes):
            ref_s, abs_s = oracle.reduce_fp(f_host, "sum", 0.0, want_abs=True)
            ref_m = oracle.reduce_fp(f_host, "max", -np.inf)
            ref_i = oracle.reduce_int(i_host, "sum", 0)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, allowed)
    step_bytes = f_host.nbytes * 2 + i_host.nbytes
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    baseline = {"value": round(passes * step_bytes / dt / 1e9, 3), "unit": "GB/s", "cores": 1,
                "kind": "oracle",
                "sample": f"{passes} serial passes of the full step (fp32 sum, fp32 max, int64 "
                          f"sum over 2^28 each; {dt:.1f} s), FP64 Neumaier sums; pinned to "
                          f"core {core}, 1 core of {len(allowed)} available ({cpu_model})"}
    return baseline, (ref_s, abs_s, ref_m, ref_i)


class OracleLeg:
    """The rest of the CPU baseline leg: the oracle on host copies of the benchmark's
    other inputs.  Its values are the references every result of the extras is checked
    against and every floating sum is reported against, as rel = |got - ref| / |ref| and
    kappa = sum|x| / |sum x| (the sum's condition number).  Absent with
    --no-cpu-baseline, when the extras report no errors."""

    def __init__(self):
        import oracle
        self.o = oracle
        self._axpy = {}

    def fp_sum(self, host, bf16=False, x0=0.0):
        """(FP64 sum, sum|x|) of a host array (bf16 as uint16 bits)."""
        return self.o.reduce_fp(host, "sum", x0, bf16=bf16, want_abs=True)

    def value(self, host, dt, op, x0):
        """(reference, sum|x| or None) of one reduction (dtype / op codes as synth's)."""
        opn = {0: "sum", 1: "max", 2: "min"}[op]
        if dt in (0, 1):
            return self.o.reduce_int(host, opn, int(x0)), None
        if op == 0:
            return self.fp_sum(host, bf16=dt == 4, x0=float(x0))
        return self.o.reduce_fp(host, opn, float(x0), bf16=dt == 4), None

    def axpy(self, torch, seed_x, seed_y, n, a=0.7):
        """Oracle of y' = fmaf(a, x, y) and its sum for the benchmark's device inputs of
        these seeds: (y' as a device tensor, sum, sum|y'|), cached."""
        key = (seed_x, seed_y, n, a)
        if key not in self._axpy:
            import synth
            xh = synth.device(synth.F32, n, seed_x).cpu().numpy()
            yh = synth.device(synth.F32, n, seed_y).cpu().numpy()
            y2, s = self.o.axpy_sum(a, xh, yh, 0.0)
            _, sabs = self.fp_sum(y2)
            self._axpy[key] = (torch.from_numpy(y2).cuda(), s, sabs)
        return self._axpy[key]

    def array_columns(self, a2d_host):
        """FP64 column sums of a row-major block."""
        import numpy as np
        return np.asarray(self.o.reduce_array(a2d_host, "sum", np.zeros(a2d_host.shape[1])))


def sum_error(got, ref, abs_sum):
    """{"rel", "kappa"} of a floating sum against its oracle value (kappa None for an
    exact sum of 0, where rel is taken against sum|x|)."""
    got, ref = float(got), float(ref)
    if ref == 0.0:
        return {"rel": abs(got) / abs_sum if abs_sum else abs(got), "kappa": None}
    return {"rel": abs(got - ref) / abs(ref), "kappa": abs_sum / abs(ref)}


MODEL_FILE = os.path.join(ROOT, "paper_2106_03219_amd", "picker_model.txt")


def _time_us(fn, torch, reps=5, inner=1):
    """Min over reps of the duration of `inner` back-to-back calls (HIP events on the
    current stream), per call, in microseconds."""
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(inner):
            fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) * 1e3 / inner)
    return best


def bench_teams_curve(om, torch, f, i, refs=None):
    """GB/s of the fp32 and int64 sums over the benchmark's 2^28 inputs against the team
    count, 1 to 2048 teams of 256 threads (static default schedule, built-in vector width
    and unroll), the runtime's default launch, and that launch with every thread reducing
    exactly its schedule(static) run (EXACT_THREAD_MAP).  With the oracle's values
    (refs = (fp32 sum, sum|x|, int64 sum)) every launch's result is checked: the int64
    sum exactly, the fp32 sum reported as rel / kappa per configuration."""
    _log("reduction GB/s against the team count")
    out = {}
    errs = {}
    exact = True
    for name, data in (("fp32_sum", f), ("int64_sum", i)):
        x = torch.zeros(1, dtype=data.dtype, device="cuda")
        row = {}
        cfgs = [(f"T={t}" if t else "default",
                 {"teams": t, "threads": 256 if t else 0, "flags": om.CFG_NO_MODEL})
                for t in [1 << k for k in range(12)] + [0]]
        # the same default launch with every thread reducing exactly its static run
        cfgs.append(("default_exact_thread_map",
                     {"flags": om.CFG_NO_MODEL | om.CFG_EXACT_THREAD_MAP}))
        for key, cfg in cfgs:
            if refs is not None:
                x.zero_()
                om.reduce(data, "sum", x, config=cfg)
                torch.cuda.synchronize()
                if name == "fp32_sum":
                    errs[key] = sum_error(x.item(), refs[0], refs[1])["rel"]
                else:
                    exact &= x.item() == refs[2]
            us = _time_us(lambda: om.reduce(data, "sum", x, config=cfg), torch, reps=3)
            row[key] = round(data.numel() * data.element_size() / us / 1e3, 1)
        out[name] = row
    if refs is not None:
        out["fp32_sum_rel_err"] = errs
        out["fp32_sum_kappa"] = refs[1] / abs(refs[0])
        out["int64_sums_exact"] = bool(exact)
        if max(errs.values()) > 1e-6 or not exact:
            _log(f"PARITY FAILURE in the team sweep: {errs} int64 exact {exact}")
            sys.exit(1)
    return out


def _axpy_check(torch, leg, y, s_val, n, what):
    """y bit for bit and the sum against the oracle: (rel, y exact), or None without it."""
    import synth
    if leg is None:
        return None
    yref, sref, sabs = leg.axpy(torch, synth.SEED_AXPY_X, synth.SEED_AXPY_Y, n)
    ok = bool(torch.equal(y.view(torch.int32), yref.view(torch.int32)))
    e = sum_error(s_val, sref, sabs)
    if not ok or e["rel"] > 1e-6:
        _log(f"PARITY FAILURE {what}: y exact {ok}, sum rel {e['rel']:.3e}")
        sys.exit(1)
    return e["rel"]


def bench_axpy(om, torch, leg=None):
    """AXPY + sum worksharing body over 2^26 fp32: chunk {0,1,64,1024} x teams x threads.

    Every schedule's y must equal the oracle's bit for bit (each iteration is one fused
    multiply-add whoever runs it) and its sum is reported against the oracle's (rel, with
    the sum's kappa); every launch of the sweep is checked the same way before it is
    timed."""
    import synth
    _log("AXPY 2^26: oracle parity and chunk x teams sweep")
    n = 1 << 26
    x = synth.device(synth.F32, n, synth.SEED_AXPY_X)
    y0 = synth.device(synth.F32, n, synth.SEED_AXPY_Y)
    y = y0.clone()
    s = torch.zeros(1, dtype=torch.float32, device="cuda")
    rels = {}

    def checked(T, P, c):
        y.copy_(y0)
        s.zero_()
        om.axpy_sum(0.7, x, y, s, T, P, 0, c)
        torch.cuda.synchronize()
        r = _axpy_check(torch, leg, y, s.item(), n, f"axpy c={c} T={T} P={P}")
        if r is not None:
            rels[f"c={c},T={T},P={P}"] = r

    table = {}
    for c in (0, 1, 64, 1024):
        for T in (64, 128, 256, 512, 1024, 2048, 4096):
            for P in (256, 512):
                checked(T, P, c)
                us = _time_us(lambda: om.axpy_sum(0.7, x, y, s, T, P, 0, c), torch)
                table[f"c={c},T={T},P={P}"] = round(12 * n / us / 1e3, 1)
        checked(0, 0, c)
        us = _time_us(lambda: om.axpy_sum(0.7, x, y, s, 0, 0, 0, c), torch)
        table[f"c={c},default"] = round(12 * n / us / 1e3, 1)
    best = {str(c): max(v for k, v in table.items() if k.startswith(f"c={c},")) for c in (0, 1, 64, 1024)}
    out = {"n": n, "bytes_per_iter": 12, "gb_s": table, "best_gb_s_per_chunk": best,
           "runtime_choice_gb_s": {str(c): table[f"c={c},default"] for c in (0, 1, 64, 1024)}}
    if leg is not None:
        out["oracle"] = {"launches_checked": len(rels), "y_bit_exact": True,
                         "sum_rel_err": rels, "sum_rel_err_max": max(rels.values()),
                         "sum_kappa": leg.axpy(torch, synth.SEED_AXPY_X, synth.SEED_AXPY_Y, n)[2]
                         / abs(leg.axpy(torch, synth.SEED_AXPY_X, synth.SEED_AXPY_Y, n)[1])}
    return out


def bench_multi(om, torch, leg=None):
    """Several reduction variables over one input: reduction(+: s) reduction(max: hi)
    reduction(min: lo) over 2^28 fp32 and int64 in one fused pass against three plain
    launches; the fused results must equal the plain ones (max, min, int64 sum exactly,
    the fp32 sum within 2e-6)."""
    _log("several reduction variables in one pass")
    out = {}
    n = 1 << 28
    for name, dt in (("fp32", torch.float32), ("int64", torch.int64)):
        g = torch.Generator(device="cuda")
        g.manual_seed(95)
        t = (torch.randn(n, device="cuda", generator=g) if dt == torch.float32 else
             torch.randint(-(2**40), 2**40, (n,), device="cuda", dtype=dt, generator=g))
        ident = {"sum": 0, "max": torch.finfo(dt).min if dt.is_floating_point else -(2**63),
                 "min": torch.finfo(dt).max if dt.is_floating_point else 2**63 - 1}
        fused = {op: torch.tensor([v], dtype=dt, device="cuda") for op, v in ident.items()}
        plain = {op: torch.tensor([v], dtype=dt, device="cuda") for op, v in ident.items()}
        om.reduce_multi(t, list(fused.items()))
        for op, x in plain.items():
            om.reduce(t, op, x)
        torch.cuda.synchronize()
        ok = all(fused[op].item() == plain[op].item() for op in ("max", "min"))
        a, b = fused["sum"].item(), plain["sum"].item()
        ok &= a == b if dt == torch.int64 else abs(a - b) <= 2e-6 * abs(b)
        errs = None
        if leg is not None:
            h = t.cpu().numpy()
            if dt == torch.int64:
                ok &= a == leg.o.reduce_int(h, "sum", 0)
            else:
                ref, sabs = leg.fp_sum(h)
                errs = {"fused": sum_error(a, ref, sabs), "plain": sum_error(b, ref, sabs)}
                ok &= max(e["rel"] for e in errs.values()) <= 1e-6
            ok &= fused["max"].item() == float(h.max()) and fused["min"].item() == float(h.min())
            del h
        us_f = _time_us(lambda: om.reduce_multi(t, list(fused.items())), torch)
        us_p = _time_us(lambda: [om.reduce(t, op, x) for op, x in plain.items()], torch)
        out[name] = {"fused_us": round(us_f, 1), "three_launches_us": round(us_p, 1),
                     "fused_gb_s": round(n * t.element_size() / us_f / 1e3, 1),
                     "speedup": round(us_p / us_f, 2), "results_agree": bool(ok)}
        if errs is not None:
            out[name]["fp32_sum_vs_oracle"] = errs
        del t
        torch.cuda.empty_cache()
    return out


def bench_loc_hist(om, torch):
    """maxloc over 2^28 fp32 (checked against torch.argmax's first occurrence) and the
    histogram of 2^28 uniform int32 keys for 256, 16 257, 100 000 and 2^20 bins, default
    strategy and atomics on hist (checked against torch.bincount), default launches."""
    _log("maxloc and histogram")
    n = 1 << 28
    g = torch.Generator(device="cuda")
    g.manual_seed(97)
    f = torch.randn(n, device="cuda", generator=g)
    val = torch.tensor([-float("inf")], device="cuda")
    idx = torch.tensor([-1], dtype=torch.int64, device="cuda")
    om.reduce_loc(f, "max", val, idx)
    torch.cuda.synchronize()
    ok = idx.item() == int(torch.argmax(f).item()) and val.item() == f.max().item()
    us = _time_us(lambda: om.reduce_loc(f, "max", val, idx), torch)
    out = {"maxloc_fp32": {"us": round(us, 1), "gb_s": round(4 * n / us / 1e3, 1), "agrees": ok}}
    del f
    out.update(bench_hist(om, torch, (256, 16257, 100000, 1 << 20), g))
    return out


def bench_hist(om, torch, bin_counts, g=None):
    """Histograms of 2^28 uniform int32 keys: the default strategy, atomics on hist
    (HIST_DIRECT) and, where they apply, range-by-range LDS copies (HIST_RANGES, up to 32
    ranges of 40 704 bins), the partition by bin range across teams (HIST_PARTITION, up to
    8 388 608 bins) and the per-tile sort by bin range (HIST_TILE_SORT, up to 4 194 304 bins),
    each checked against torch.bincount."""
    n = 1 << 28
    if g is None:
        g = torch.Generator(device="cuda")
        g.manual_seed(97)
    out = {}
    for bins in bin_counts:
        k = torch.randint(0, bins, (n,), device="cuda", dtype=torch.int32, generator=g)
        want = torch.bincount(k.long(), minlength=bins)
        h = torch.zeros(bins, dtype=torch.int32, device="cuda")
        forms = [("", None), ("_direct", {"flags": om.CFG_HIST_DIRECT})]
        if 40704 < bins <= 32 * 40704:
            forms.append(("_ranges", {"flags": om.CFG_HIST_RANGES}))
        if 40704 < bins <= 8388608:
            forms.append(("_partition", {"flags": om.CFG_HIST_PARTITION}))
        if 40704 < bins <= 128 * 32768:
            forms.append(("_tile_sort", {"flags": om.CFG_HIST_TILE_SORT}))
        for name, cfg in forms:
            h.zero_()
            om.histogram(k, bins, h, config=cfg)
            torch.cuda.synchronize()
            agrees = bool(torch.equal(h.long(), want))
            us = _time_us(lambda: om.histogram(k, bins, h, config=cfg), torch, reps=3)
            out[f"histogram_{bins}_bins{name}"] = {"us": round(us, 1),
                                                   "gkeys_s": round(n / us / 1e3, 3),
                                                   "agrees": agrees}
        del k, want
        torch.cuda.empty_cache()
    return out


def bench_generic(om, torch):
    """The generic-mode region (power iteration on a diagonal matrix, 100 steps) with one
    team of 1024 threads, with the default co-resident teams, and for 2^20 elements a sweep
    of team counts, against the same region written as one launch per parallel loop
    (torch: multiply, dot, rsqrt, scale; four launches a step).  Per step the loops move
    20 bytes an element (read d and v, write v; read and write v).  Each form's v must
    agree with the per-loop form's to 1e-4."""
    import synth
    _log("generic-mode power iteration")
    out = {}
    iters = 100
    for n in (1 << 12, 1 << 16, 1 << 20, 1 << 24):
        dh, vh = synth.power_inputs(n, 11)
        d = torch.from_numpy(dh).cuda()
        v0 = torch.from_numpy(vh).cuda()
        w = v0.clone()
        s = torch.zeros((), device="cuda")

        def per_loop():
            for _ in range(iters):
                torch.mul(d, w, out=w)
                torch.dot(w, w, out=s)
                w.mul_(torch.rsqrt(s))

        per_loop()
        torch.cuda.synchronize()
        want = w.clone()
        us_t = _time_us(per_loop, torch, reps=3)
        row = {"launch_per_loop_us_per_step": round(us_t / iters, 2)}
        v = v0.clone()
        lam = torch.zeros(1, device="cuda")
        shapes = [("one_team", 1, 1024), ("default", 0, 0)]
        if n == 1 << 20:
            shapes += [(f"{t}x{p}", t, p) for t in (64, 128, 256, 512) for p in (256, 1024)]
        for name, teams, threads in shapes:
            if n == 1 << 24 and teams == 1:
                continue
            v.copy_(v0)
            om.generic_power(d, v, iters, lam, teams, threads)
            torch.cuda.synchronize()
            agrees = bool(torch.allclose(v, want, rtol=1e-4, atol=1e-12))
            us = _time_us(lambda: om.generic_power(d, v, iters, lam, teams, threads), torch, reps=3)
            row[name] = {"us_per_step": round(us / iters, 2), "gb_s": round(20 * n * iters / us / 1e3, 1),
                         "speedup_vs_per_loop": round(us_t / us, 2), "agrees": agrees}
        out[f"n_{n}"] = row
        del d, v0, w, v, want
        torch.cuda.empty_cache()
    return out


def bench_region(om, torch, leg=None):
    """The two-loop region over 2^26 fp32 (AXPY loop, then the sum loop over the updated y)
    with and without the barrier between the loops, next to the fused body that does both
    in one loop; default teams and threads, chunks 0, 1 and 64.  The loops move 16 bytes an
    element (the fused body 12).  y must be bit-identical to the fused body's and the sums
    within 2e-6 of it."""
    import synth
    _log("two-loop region over 2^26 with and without nowait")
    n = 1 << 26
    x = synth.device(synth.F32, n, synth.SEED_AXPY_X)
    y0 = synth.device(synth.F32, n, synth.SEED_AXPY_Y)
    y = y0.clone()
    s = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = {}
    for c in (0, 1, 64):
        yref = y0.clone()
        sref = torch.zeros(1, dtype=torch.float32, device="cuda")
        om.axpy_sum(0.7, x, yref, sref, 0, 0, 0, c)
        row = {}
        forms = (("fused", lambda: om.axpy_sum(0.7, x, y, s, 0, 0, 0, c), 12),
                 ("barrier", lambda: om.region_axpy_sum(0.7, x, y, s, 0, 0, 0, c, c, False), 16),
                 ("nowait", lambda: om.region_axpy_sum(0.7, x, y, s, 0, 0, 0, c, c, True), 16))
        for name, fn, bpe in forms:
            y.copy_(y0)
            s.zero_()
            fn()
            torch.cuda.synchronize()
            agrees = bool(torch.equal(y, yref)) and abs(s.item() - sref.item()) <= 2e-6 * abs(sref.item())
            rel = _axpy_check(torch, leg, y, s.item(), n, f"region {name} c={c}")
            us = _time_us(fn, torch)
            row[name] = {"us": round(us, 1), "gb_s": round(bpe * n / us / 1e3, 1), "agrees": agrees}
            if rel is not None:
                row[name]["sum_rel_err_vs_oracle"] = rel
        out[f"chunk_{c}"] = row
    return out


def bench_udr(om, torch):
    """User-defined reductions (declared at run time, compiled by hiprtc) over 2^28
    elements, default launch: Welford's count / mean / M2 over fp32 (checked against
    torch.var_mean, and timed beside it), an exact three-field integer reduction over int32,
    and a 16-bin histogram type (64 bytes) over int64."""
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    import udr_cases as U
    import synth
    _log("user-defined reductions")
    n = 1 << 28
    out = {}
    for name, dtype in (("WELFORD", synth.F32), ("STATS3", synth.I32), ("HIST16", synth.I64)):
        c = getattr(U, name)
        t0 = time.time()
        h = om.udr_declare(c["type_def"], c["initializer"], c["combiner"], c["body"],
                           c["acc_bytes"], dtype)
        compile_s = time.time() - t0
        data = synth.device(dtype, n, 91)
        x0 = torch.from_numpy(U.pack(name, getattr(U, name.lower() + "_init")())).cuda()
        x = x0.clone()

        def fn():
            x.copy_(x0)
            om.reduce_udr(h, data, x)

        us = _time_us(fn, torch)
        row = {"us": round(us, 1), "gb_s": round(n * data.element_size() / us / 1e3, 1),
               "declare_compile_s": round(compile_s, 2)}
        if name == "WELFORD":
            fn()
            torch.cuda.synchronize()
            cnt, mean, m2 = U.unpack(name, x.cpu().numpy())
            var_t, mean_t = torch.var_mean(data, correction=0)
            row["agrees_with_torch_var_mean"] = bool(
                cnt == n and abs(mean - mean_t.item()) <= 1e-5 * (abs(mean_t.item()) + var_t.item() ** 0.5)
                and abs(m2 / n - var_t.item()) <= 1e-5 * var_t.item())
            us_t = _time_us(lambda: torch.var_mean(data, correction=0), torch)
            row["torch_var_mean_us"] = round(us_t, 1)
        out[name.lower()] = row
        del data
        torch.cuda.empty_cache()
    return out


def bench_queue(om, torch, leg=None):
    """The AXPY + sum body over 2^26 fp32 under schedule(dynamic, c) and schedule(guided,
    c) for the threads of each team (distribute static, one team per compute unit, 512
    threads, and the runtime's default team size), next to the static schedule with the
    same chunk.  y must be bit-identical to
    the static schedule's and the sums within 2e-6 of it."""
    import synth
    _log("AXPY 2^26 under dynamic / guided schedules")
    n = 1 << 26
    x = synth.device(synth.F32, n, synth.SEED_AXPY_X)
    y0 = synth.device(synth.F32, n, synth.SEED_AXPY_Y)
    yref = y0.clone()
    sref = torch.zeros(1, dtype=torch.float32, device="cuda")
    om.axpy_sum(0.7, x, yref, sref)
    torch.cuda.synchronize()
    y = y0.clone()
    s = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = {}
    rels = {}
    agree = True
    for kind, c in (("static", 0), ("static", 1), ("static", 64), ("static", 1024),
                    ("dynamic", 1), ("dynamic", 4), ("dynamic", 64), ("dynamic", 1024),
                    ("guided", 1), ("guided", 64)):
        if kind == "static":
            fn = lambda: om.axpy_sum(0.7, x, y, s, 0, 512, 0, c)
        else:
            fn = lambda: om.axpy_sum_queue(kind, 0.7, x, y, s, 0, 512, 0, c)
        y.copy_(y0)
        s.zero_()
        fn()
        torch.cuda.synchronize()
        agree &= bool(torch.equal(y, yref))
        agree &= abs(s.item() - sref.item()) <= 2e-6 * abs(sref.item())
        rel = _axpy_check(torch, leg, y, s.item(), n, f"queue {kind} c={c}")
        if rel is not None:
            rels[f"{kind},c={c}"] = rel
        us = _time_us(fn, torch)
        out[f"{kind},c={c}"] = round(12 * n / us / 1e3, 1)
        if kind != "static":   # the runtime's own team size (threads 0)
            fd = lambda: om.axpy_sum_queue(kind, 0.7, x, y, s, 0, 0, 0, c)
            y.copy_(y0)
            s.zero_()
            fd()
            torch.cuda.synchronize()
            agree &= bool(torch.equal(y, yref))
            agree &= abs(s.item() - sref.item()) <= 2e-6 * abs(sref.item())
            us = _time_us(fd, torch)
            out[f"{kind},c={c},default_threads"] = round(12 * n / us / 1e3, 1)
    res = {"n": n, "bytes_per_iter": 12, "gb_s": out, "y_and_sum_agree_with_static": agree}
    if rels:
        res["sum_rel_err_vs_oracle"] = rels
    return res


def bench_latency(om, torch):
    """Launch latency of empty target regions and tiny reductions."""
    import statistics
    _log("launch latency sweep")
    res = {}
    stream = torch.cuda.current_stream()
    for n in (0, 1, 16, 1024):
        for T in (1, 64):
            k = 2000
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                om.empty_region(n, T, 256)
            t1 = time.perf_counter()
            torch.cuda.synchronize()
            b2b = _time_us(lambda: om.empty_region(n, T, 256), torch, reps=3, inner=k)
            rt = []
            for _ in range(200):
                t2 = time.perf_counter()
                om.empty_region(n, T, 256)
                torch.cuda.synchronize()
                rt.append((time.perf_counter() - t2) * 1e6)
            res[f"empty n={n} T={T}"] = {"host_enqueue_us": round((t1 - t0) / k * 1e6, 2),
                                         "back_to_back_us": round(b2b, 2),
                                         "round_trip_us": round(statistics.median(rt), 2)}
    a = torch.ones(1024, dtype=torch.int32, device="cuda")
    x = torch.zeros(1, dtype=torch.int32, device="cuda")
    for n in (1, 1024):
        b2b = _time_us(lambda: om.reduce(a[:n], "sum", x), torch, reps=3, inner=2000)
        rt = []
        for _ in range(200):
            t2 = time.perf_counter()
            om.reduce(a[:n], "sum", x)
            torch.cuda.synchronize()
            rt.append((time.perf_counter() - t2) * 1e6)
        res[f"reduce int32 n={n}"] = {"back_to_back_us": round(b2b, 2),
                                      "round_trip_us": round(statistics.median(rt), 2)}
    # host cost without Python: 4096 one-element reductions issued from C in one call
    ones = torch.ones(4096, dtype=torch.int64, device="cuda")
    outs = torch.zeros(4096, dtype=torch.int64, device="cuda")
    segs = om.make_segments([(ones[k:k + 1], "sum", outs[k:k + 1]) for k in range(4096)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    om.reduce_each(segs, config={"flags": om.CFG_NO_MODEL})
    t1 = time.perf_counter()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    res["4096 plain 1-element reductions issued from C"] = {
        "host_enqueue_us_per_launch": round((t1 - t0) / 4096 * 1e6, 2),
        "completion_us_per_launch": round((t2 - t0) / 4096 * 1e6, 2)}
    # graph replay: 100 empty regions captured once on a side stream
    s = torch.cuda.Stream()
    om.workspace_reserve(64, stream=s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(100):
            om.empty_region(16, 1, 256)
    g.replay()
    torch.cuda.synchronize()
    rep = _time_us(lambda: g.replay(), torch, reps=5, inner=10)
    res["graph replay of 100 empty regions: us per region"] = round(rep / 100, 3)
    del stream
    return res


def _identity(om, dt, op):
    import numpy as np
    if op == "sum":
        return 0
    if dt in (om.I32, om.I64):
        info = np.iinfo(np.int32 if dt == om.I32 else np.int64)
        return int(info.min if op == "max" else info.max)
    return float("-inf") if op == "max" else float("inf")


def bench_batched(om, torch, leg=None):
    """4096 independent reductions (lengths log-uniform 1e2..1e7, int64/fp32/bf16, sum/max/min):
    4096 plain launches (heuristic / learned configuration) vs one graph-replayed persistent
    launch (default tiles / autotuned tiles).  With the oracle leg, every segment of every
    form is checked against the oracle (integers and max/min exactly, floating sums within
    1e-6) and the floating sums' errors are reported per dtype (max and median rel, with
    the kappa of the worst); the oracle's own time over the 4096 segments is the CPU
    figure."""
    import statistics

    import numpy as np

    import synth
    _log("batched: generating 4096 segments")
    lens, dts, ops = synth.batched_spec(4096, synth.SEED_BATCH)
    opn = {0: "sum", 1: "max", 2: "min"}
    tdt = {om.I32: torch.int32, om.I64: torch.int64, om.F32: torch.float32, om.F64: torch.float64,
           om.BF16: torch.bfloat16}
    ins = [synth.device(int(dts[k]), int(lens[k]), 20_000 + k) for k in range(4096)]
    meta = [(int(dts[k]), int(ops[k])) for k in range(4096)]
    xs = []
    for dt, op in meta:
        xdt = torch.float32 if (dt == om.BF16 and op == 0) else tdt[dt]
        xs.append(torch.tensor([_identity(om, dt, opn[op])], dtype=xdt, device="cuda"))
    x0 = [x.clone() for x in xs]
    segs = om.make_segments([(t, opn[op], x) for t, x, (dt, op) in zip(ins, xs, meta)])
    total_bytes = int(sum(t.numel() * t.element_size() for t in ins))
    i64_idx = [k for k, x in enumerate(xs) if x.dtype == torch.int64]
    fp_idx = [k for k, x in enumerate(xs) if x.dtype != torch.int64]   # exact in float64
    got = {}

    def check(name, run):
        for x, v in zip(xs, x0):
            x.copy_(v)
        run()
        torch.cuda.synchronize()
        vi = torch.cat([xs[k].view(-1) for k in i64_idx]).cpu().tolist() if i64_idx else []
        vf = torch.cat([xs[k].view(-1).double() for k in fp_idx]).cpu().tolist() if fp_idx else []
        res = [None] * len(xs)
        for k, v in zip(i64_idx, vi):
            res[k] = int(v)
        for k, v in zip(fp_idx, vf):
            res[k] = float(v)
        got[name] = res

    results, times = {}, {}

    def measure(name, run):
        check(name, run)
        us = _time_us(run, torch, reps=3)
        times[name] = us
        results[name] = {"ms": round(us / 1e3, 3), "reductions_per_s": round(4096 / (us * 1e-6), 1),
                         "gb_s": round(total_bytes / us / 1e3, 1)}
        _log(f"batched {name}: {us / 1e3:.3f} ms")

    measure("plain_heuristic", lambda: om.reduce_each(segs, config={"flags": om.CFG_NO_MODEL}))
    if os.path.exists(MODEL_FILE):
        om.model_load(MODEL_FILE)
        measure("plain_learned", lambda: om.reduce_each(segs))
        om.model_load(None)
    measure("batched_graph", lambda: om.reduce_batched(segs))
    sweep = {}
    for tk in (64, 256, 1024, 4096):
        for th in (256, 512, 1024):
            cfg = {"tile_kib": tk, "threads": th}
            us = _time_us(lambda: om.reduce_batched(segs, config=cfg), torch, reps=3)
            sweep[f"tile={tk}KiB,threads={th}"] = round(us / 1e3, 3)
    best = min(sweep, key=sweep.get)
    tk, th = [int(v.split("=")[1].rstrip("KiB")) for v in best.split(",")]
    measure("batched_graph_tuned", lambda: om.reduce_batched(segs, config={"tile_kib": tk, "threads": th}))
    results["batched_graph_tuned"]["config"] = {"tile_kib": tk, "threads": th}
    out = {"segments": 4096, "bytes": total_bytes, "forms": results,
           "tile_sweep_ms": sweep,
           "reductions_per_s": {k: v["reductions_per_s"] for k, v in results.items()}}
    if "plain_learned" in times:
        out["learned_vs_plain_speedup"] = round(times["plain_heuristic"] / times["plain_learned"], 3)
    out["batched_vs_plain_speedup"] = round(times["plain_heuristic"] / times["batched_graph_tuned"], 2)
    if leg is not None:
        _log("batched: the oracle over all 4096 segments (host copies, one core)")
        refs, t_oracle = [], 0.0
        for k, (dt, op) in enumerate(meta):
            t = ins[k]
            h = t.view(torch.int16).cpu().numpy().view(np.uint16) if t.dtype == torch.bfloat16 \
                else t.cpu().numpy()
            ident = _identity(om, dt, opn[op])
            t0 = time.perf_counter()
            refs.append(leg.value(h, dt, op, ident))
            t_oracle += time.perf_counter() - t0
        out["oracle_cpu"] = {"seconds": round(t_oracle, 2), "cores": 1,
                             "reductions_per_s": round(4096 / t_oracle, 1),
                             "gb_s": round(total_bytes / t_oracle / 1e9, 3)}
        failed = False
        for name, res in got.items():
            match, errs = 0, {"f32": [], "bf16": []}
            for k, ((dt, op), v, (ref, sabs)) in enumerate(zip(meta, res, refs)):
                if op == 0 and dt in (om.F32, om.BF16):
                    e = sum_error(v, ref, sabs)
                    errs["f32" if dt == om.F32 else "bf16"].append((e["rel"], e["kappa"], k))
                    match += e["rel"] <= 1e-6
                else:
                    match += v == ref
            rep = {"segments_matching": match, "segments": 4096}
            for dn, lst in errs.items():
                if lst:
                    worst = max(lst)
                    rep[f"{dn}_sum"] = {"results": len(lst), "rel_max": worst[0],
                                        "rel_median": statistics.median(r for r, _, _ in lst),
                                        "kappa_at_max": worst[1], "segment_at_max": worst[2],
                                        "kappa_max": max((kk for _, kk, _ in lst if kk), default=None)}
            results[name]["oracle"] = rep
            failed |= match != 4096
        if failed:
            _log("PARITY FAILURE in the batched workload: " +
                 str({n: r["oracle"]["segments_matching"] for n, r in results.items()}))
            sys.exit(1)
    del ins
    torch.cuda.empty_cache()
    return out


def bench_atomics(om, torch):
    """Throughput of the five device atomics: 2^24 operations, uncontended (one word
    each), on 256 words, and all on one word."""
    _log("device atomics throughput")
    n = 1 << 24
    e = torch.ones(n, dtype=torch.int32, device="cuda")
    d = torch.zeros(n, dtype=torch.int32, device="cuda")
    old = torch.empty(n, dtype=torch.int32, device="cuda")
    out = {}
    for name, words in (("uncontended", n), ("256_words", 256), ("one_word", 1)):
        target = torch.zeros(words, dtype=torch.int32, device="cuda")
        index = (torch.arange(n, device="cuda", dtype=torch.int64) % words).to(torch.int32)
        row = {}
        for op in ("add", "inc", "max", "exchange", "cas"):
            us = _time_us(lambda: om.atomic_apply(op, target, index, e, old, d=d), torch, reps=3)
            row[op] = round(n / us / 1e3, 2)
        out[name] = row
    return {"ops": n, "gops_per_s": out}


def bench_array(om, torch, leg=None):
    """Array-section reductions reduction(+: x[0:m]) over 2^28-element row-major blocks
    (1 GiB fp32, 2 GiB int64) in the runtime's default launch: GB/s of the input read
    per launch, the same data's plain reduction for scale, and a check of every column
    against torch's column sums (int64 exact, fp32 within 1e-6 of an fp64 sum)."""
    _log("array-section reductions")
    out = []
    n = 1 << 28
    for rows, m, dt in ((n // 8, 8, torch.float32), (n // 4096, 4096, torch.float32),
                        (n >> 20, 1 << 20, torch.float32), (n // 8, 8, torch.int64)):
        g = torch.Generator(device="cuda")
        g.manual_seed(90 + m)
        if dt == torch.int64:
            inp = torch.randint(-(2**40), 2**40, (n,), device="cuda", dtype=dt, generator=g)
        else:
            inp = torch.randn(n, device="cuda", dtype=dt, generator=g)
        x = torch.zeros(m, dtype=dt, device="cuda")
        us = _time_us(lambda: om.reduce_array(inp, rows, m, "sum", x), torch, reps=5)
        xs = torch.zeros(1, dtype=dt, device="cuda")
        us_plain = _time_us(lambda: om.reduce(inp, "sum", xs), torch, reps=5)
        x.zero_()
        om.reduce_array(inp, rows, m, "sum", x)
        rel = None
        if leg is not None and dt == torch.float32 and m <= 4096:
            hv = inp.view(rows, m).cpu().numpy()
            ref = torch.from_numpy(leg.array_columns(hv)).cuda()
            del hv
            err = (x.double() - ref).abs()
            rel = float((err / ref.abs()).max())
            ok = bool((err <= 1e-6 * ref.abs()).all())
        else:
            ref = inp.view(rows, m).sum(dim=0, dtype=torch.float64 if dt == torch.float32 else dt)
            if dt == torch.int64:
                ok = bool(torch.equal(x, ref))
            else:
                ok = bool(((x.double() - ref).abs() <= 1e-6 * ref.abs() + 1e-6).all())
        plan = om.reduce_array_plan(rows, m, om.dtype_code(inp), "sum")
        out.append({"rows": rows, "m": m, "dtype": str(dt).replace("torch.", ""),
                    "us": round(us, 1), "gb_per_s": round(n * inp.element_size() / us / 1e3, 1),
                    "plain_reduction_gb_per_s": round(n * inp.element_size() / us_plain / 1e3, 1),
                    "tiles": plan[2], "row_teams": plan[3], "groups": plan[4], "columns_ok": ok})
        if rel is not None:
            out[-1]["column_sum_rel_err_max_vs_oracle"] = rel
        if not ok:
            _log(f"ARRAY COLUMN MISMATCH rows={rows} m={m} {dt}")
            sys.exit(1)
        del inp, ref
        torch.cuda.empty_cache()
    return out


def bench_learned(om, torch, count=300):
    """The learned picker on a sample of the held-out instance distribution (seed 8,
    n <= 1e8): total and geometric-mean time with the model's launches vs the built-in
    heuristic's, each timed as the autotuner times its classes (GPU time a launch adds to
    a stream of launches over inputs not in cache; min of 2 batches); both launches of an
    instance must agree (identical integer/max/min results, sums within 2e-6)."""
    import math

    import synth
    from paper_2106_03219_amd.tune import Windows, calibrate_spin, time_call
    if not os.path.exists(MODEL_FILE):
        return None
    _log(f"learned picker: {count} held-out instances, model vs heuristic")
    inst = synth.cost_instances(2 * count, synth.SEED_HELDOUT)
    keep = [i for i in range(2 * count) if inst["n"][i] <= 10**8][:count]
    nmax = int(max(inst["n"][i] for i in keep))
    bufs = {dt: synth.device(dt, nmax, 60 + dt) for dt in (om.I32, om.I64, om.F32, om.BF16)}
    ybuf = synth.device(om.F32, nmax, 70)
    opn = {0: "sum", 1: "max", 2: "min"}
    calibrate_spin(torch)
    cursor = [0]
    om.model_load(MODEL_FILE)
    t_model = t_heur = 0.0
    logs = 0.0
    agree = True
    picked = 0
    try:
        for i in keep:
            n, dt, op, body, ch = (int(inst[k][i]) for k in ("n", "dtype", "op", "body", "chunk"))
            res = []
            tt = []
            ebytes = 12 if body else {om.I32: 4, om.I64: 8, om.F32: 4, om.BF16: 2}[dt]
            win = Windows(cursor, n, nmax, 3 if n * ebytes > (64 << 20) else 8)
            for cfg in (None, {"flags": om.CFG_NO_MODEL}):
                if body:
                    xb, yb = bufs[om.F32], ybuf
                    s = torch.zeros(1, dtype=torch.float32, device="cuda")
                    fn = lambda o: om.axpy_sum(0.7, xb[o:o + n], yb[o:o + n], s, 0, 0, 0,
                                               max(ch, 0), config=cfg)
                    tt.append(time_call(fn, 2, torch, win))
                    res.append(None)
                else:
                    full = bufs[dt]
                    inp = full[:n]
                    xdt = torch.float32 if (dt == om.BF16 and op == 0) else inp.dtype
                    xo = torch.tensor([_identity(om, dt, opn[op])], dtype=xdt, device="cuda")
                    om.reduce(inp, opn[op], xo, config=cfg)
                    torch.cuda.synchronize()
                    res.append(float(xo.float().item()) if xo.dtype == torch.bfloat16 else xo.item())
                    tt.append(time_call(lambda o: om.reduce(full[o:o + n], opn[op], xo, config=cfg),
                                        2, torch, win))
            _, src = om.resolve_config(n, dt, op, body, max(ch, 0) if body else -1)
            picked += src == 1
            if res[0] is not None:
                if op == 0 and dt in (om.F32, om.BF16):
                    agree &= abs(res[0] - res[1]) <= 2e-6 * max(abs(res[1]), 1e-30)
                else:
                    agree &= res[0] == res[1]
            t_model += tt[0]
            t_heur += tt[1]
            logs += math.log(tt[1] / tt[0])
    finally:
        om.model_load(None)
    del bufs, ybuf
    torch.cuda.empty_cache()
    return {"instances": len(keep), "model_decided": picked,
            "total_ms_learned": round(t_model / 1e3, 3), "total_ms_heuristic": round(t_heur / 1e3, 3),
            "total_time_speedup": round(t_heur / t_model, 3),
            "geomean_speedup": round(math.exp(logs / len(keep)), 3),
            "results_agree": bool(agree)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-passes", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the AXPY, latency, batched, atomics, array and picker measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 3 device copies of 2^28 fp32 (1 GiB read + 1 GiB written), "
                         "the reference for scaling HBM byte counters")
    ap.add_argument("--only-axpy", type=int, nargs=2, metavar=("TEAMS", "CHUNK"), default=None,
                    help="only run 3 AXPY+sum launches over 2^26 with --threads threads "
                         "(profiling)")
    ap.add_argument("--threads", type=int, default=256,
                    help="threads per team of --only-axpy (default 256)")
    ap.add_argument("--only-exact", action="store_true",
                    help="only run 3 fp32 and 3 int64 sums over 2^28 with every thread reducing "
                         "exactly its schedule(static) run, default launch (profiling)")
    ap.add_argument("--only-queue", nargs=2, metavar=("KIND", "CHUNK"), default=None,
                    help="only run 3 AXPY+sum launches over 2^26 under schedule(KIND, CHUNK), "
                         "KIND dynamic or guided, default teams x 512 threads (profiling)")
    ap.add_argument("--only-array", action="store_true",
                    help="only run the array-section reduction measurements (profiling)")
    ap.add_argument("--only-generic", action="store_true",
                    help="only run the generic-mode power iteration measurements")
    ap.add_argument("--only-region", action="store_true",
                    help="only run the two-loop region (nowait) measurements")
    ap.add_argument("--only-udr", action="store_true",
                    help="only run the user-defined reduction measurements")
    ap.add_argument("--only-batched", action="store_true",
                    help="only run the batched workload (4096 segments), its forms checked "
                         "against the oracle")
    ap.add_argument("--only-hist", action="store_true",
                    help="only run the histogram strategy sweep over bin counts")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the kernels run on one GPU and the figure is that GPU's throughput; the "
              "multi-GPU exchange is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2106_03219_amd as om
    om.load()
    torch.cuda.set_device(0)
    try:
        run(args, om, torch)
    finally:
        om.finalize()   # release the library's device memory before the runtime shuts down


def run(args, om, torch):
    import numpy as np

    import synth
    stream = torch.cuda.current_stream()

    if args.only_axpy:
        teams, chunk = args.only_axpy
        x = synth.device(synth.F32, 1 << 26, synth.SEED_AXPY_X)
        y = synth.device(synth.F32, 1 << 26, synth.SEED_AXPY_Y)
        s = torch.zeros(1, dtype=torch.float32, device="cuda")
        for _ in range(3):
            om.axpy_sum(0.7, x, y, s, teams, args.threads, 0, chunk)
        torch.cuda.synchronize()
        _log(f"3 AXPY+sum launches over 2^26, {teams} teams x {args.threads} threads, "
             f"chunk {chunk}")
        return

    if args.only_exact:
        for dt, seed in ((synth.F32, synth.SEED_F32), (synth.I64, synth.SEED_I64)):
            t = synth.device(dt, N, seed)
            x = torch.zeros(1, dtype=t.dtype, device="cuda")
            for _ in range(3):
                om.reduce(t, "sum", x, config={"flags": om.CFG_EXACT_THREAD_MAP})
            torch.cuda.synchronize()
            del t
        _log("3 fp32 and 3 int64 exact-map sums over 2^28, default launch")
        return

    if args.only_queue:
        kind, chunk = args.only_queue[0], int(args.only_queue[1])
        x = synth.device(synth.F32, 1 << 26, synth.SEED_AXPY_X)
        y = synth.device(synth.F32, 1 << 26, synth.SEED_AXPY_Y)
        s = torch.zeros(1, dtype=torch.float32, device="cuda")
        for _ in range(3):
            om.axpy_sum_queue(kind, 0.7, x, y, s, 0, 512, 0, chunk)
        torch.cuda.synchronize()
        _log(f"3 AXPY+sum launches over 2^26, schedule({kind}, {chunk}), 512 threads")
        return

    if args.only_array:
        print(json.dumps({"array_reduction": bench_array(om, torch)}), flush=True)
        return

    if args.only_generic:
        print(json.dumps({"generic_power": bench_generic(om, torch)}), flush=True)
        return

    if args.only_region:
        print(json.dumps({"region_two_loops": bench_region(om, torch)}), flush=True)
        return

    if args.only_udr:
        print(json.dumps({"user_defined_reductions": bench_udr(om, torch)}), flush=True)
        return

    if args.only_batched:
        print(json.dumps({"batched": bench_batched(om, torch, OracleLeg())}), flush=True)
        return

    if args.only_hist:
        bins = (256, 4096, 16257, 40704, 40705, 81409, 100000, 260096, 1 << 20, 1302529, 1 << 21,
                1 << 22, 1 << 23, 1 << 24)
        print(json.dumps({"histogram": bench_hist(om, torch, bins)}), flush=True)
        return

    if args.calibrate_copy:
        src = torch.ones(N, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log("copy calibration done: 3 x 1 GiB device copies")
        return

    _log("generating inputs on the device")
    f = synth.device(synth.F32, N, synth.SEED_F32)
    i = synth.device(synth.I64, N, synth.SEED_I64)
    xs = torch.zeros(1, dtype=torch.float32, device="cuda")
    xm = torch.full((1,), -float("inf"), dtype=torch.float32, device="cuda")
    xi = torch.zeros(1, dtype=torch.int64, device="cuda")
    cfg_f, _ = om.resolve_config(N, om.F32, "sum")
    cfg_i, _ = om.resolve_config(N, om.I64, "sum")

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        om.reduce(i, "sum", xi)
        if ev is not None:
            ev[1].record(stream)
        om.reduce(f, "sum", xs)
        om.reduce(f, "max", xm)

    # one untimed step whose results the CPU baseline leg checks below
    xs.zero_(); xm.fill_(-float("inf")); xi.zero_()
    step()
    torch.cuda.synchronize()
    got = (xs.item(), xm.item(), xi.item())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    _log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_bytes = f.numel() * 4 * 2 + i.numel() * 8
    value = args.steps * step_bytes / dt / 1e9
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    achieved = i.numel() * 8 / (kern_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(),
                "kernel": "omprt::reduce_kernel<1, 0, 16, 4> (int64 sum)", "avg_launch_us": round(kern_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": i.numel() * 8}

    # references on the same data: torch's own reductions and a device copy
    refs = {}
    us = _time_us(lambda: torch.sum(i), torch)
    refs["torch_sum_int64_gb_s"] = round(i.numel() * 8 / us / 1e3, 1)
    us = _time_us(lambda: torch.sum(f), torch)
    refs["torch_sum_fp32_gb_s"] = round(f.numel() * 4 / us / 1e3, 1)
    us = _time_us(lambda: torch.amax(f), torch)
    refs["torch_amax_fp32_gb_s"] = round(f.numel() * 4 / us / 1e3, 1)
    dst = torch.empty_like(f)
    us = _time_us(lambda: dst.copy_(f), torch)
    refs["torch_copy_fp32_gb_s"] = round(2 * f.numel() * 4 / us / 1e3, 1)   # read + write
    del dst
    roofline["int64_sum_vs_torch_sum"] = round(achieved / refs["torch_sum_int64_gb_s"], 3)
    roofline["int64_sum_vs_torch_copy"] = round(achieved / refs["torch_copy_fp32_gb_s"], 3)

    cpu, parity, leg, refs_c2 = None, None, None, None
    if not args.no_cpu_baseline:
        _log("CPU baseline leg: timing the oracle on the same step, checking the GPU step")
        cpu, (ref_s, abs_s, ref_m, ref_i) = cpu_baseline(f.cpu().numpy(), i.cpu().numpy(),
                                                         args.cpu_passes)
        rel = abs(got[0] - ref_s) / abs(ref_s)
        parity = {"fp32_sum_rel_err": rel, "fp32_sum_kappa": abs_s / abs(ref_s),
                  "fp32_max_exact": got[1] == ref_m, "int64_sum_exact": got[2] == ref_i}
        if not (rel <= 1e-6 and parity["fp32_max_exact"] and parity["int64_sum_exact"]):
            _log(f"PARITY FAILURE {parity}")
            sys.exit(1)
        leg = OracleLeg()
        refs_c2 = (ref_s, abs_s, ref_i)

    extra = {}
    if not args.no_extras:
        extra["teams_curve"] = bench_teams_curve(om, torch, f, i, refs_c2)
        del f, i
        torch.cuda.empty_cache()
        extra["axpy"] = bench_axpy(om, torch, leg)
        extra["latency"] = bench_latency(om, torch)
        extra["batched"] = bench_batched(om, torch, leg)
        extra["atomics"] = bench_atomics(om, torch)
        extra["array_reduction"] = bench_array(om, torch, leg)
        extra["queue_schedules"] = bench_queue(om, torch, leg)
        extra["several_variables"] = bench_multi(om, torch, leg)
        extra["maxloc_histogram"] = bench_loc_hist(om, torch)
        extra["generic_power"] = bench_generic(om, torch)
        extra["region_two_loops"] = bench_region(om, torch, leg)
        extra["user_defined_reductions"] = bench_udr(om, torch)
        learned = bench_learned(om, torch)
        if learned is not None:
            extra["learned_picker_heldout"] = learned

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32,i64",
        "data": "synthetic",
        "config": {"workload": "plain reductions at scale: fp32 sum + fp32 max over 2^28 N(0,1), "
                               "int64 sum over 2^28 U[-2^40,2^40]; static team blocks",
                   "n": N, "bytes_per_step": step_bytes,
                   "launch_fp32": cfg_f, "launch_int64": cfg_i},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "parity": parity,
        "roofline": roofline,
        "reference_kernels": refs,
        "cpu_baseline": cpu,
    }
    if "batched" in extra:
        out["batched_reductions_per_s"] = extra["batched"]["reductions_per_s"]
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
