"""omprt -- the data-parallel core of an OpenMP device runtime on MI355X.

Thin Python binding of libomprt.so (include/omprt.h): argument marshalling
only.  Every step runs in the library's HIP kernels; torch is used for
device memory and streams.  Functions keep the C names without the
``omprt_`` prefix.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (ATOMIC_ADD, ATOMIC_CAS, ATOMIC_EXCHANGE, ATOMIC_INC, ATOMIC_MAX, BAND, BF16,
                   BOR, BXOR, CFG_EXACT_THREAD_MAP, CFG_HIST_DIRECT, CFG_HIST_PARTITION, CFG_HIST_RANGES, CFG_HIST_TEAM_COPY, CFG_HIST_TILE_SORT, CFG_NO_MODEL, CFG_STATIC_TILES, F32, F64, I32, I64, LAND, LOR, MAX,
                   MIN, PROD, SUM, Config, MlpDims, OmprtError, Sched, Segment, check)

__all__ = [
    "load", "version", "for_static_bounds", "sched_count", "static_map", "reduce",
    "reduce_batched", "reduce_each", "make_segments", "axpy_sum", "empty_region", "atomic_apply",
    "ATOMIC_ADD", "ATOMIC_INC", "ATOMIC_MAX", "ATOMIC_EXCHANGE", "ATOMIC_CAS",
    "mlp_param_count", "mlp_forward", "mlp_loss_grad", "mlp_adam", "mlp_adam_counted", "model_load",
    "model_features", "resolve_config", "tune_set", "workspace_reserve", "workspace_reset",
    "workspace_status", "finalize", "reduce_noalloc", "dtype_code", "OmprtError", "Config", "Sched", "Segment", "MlpDims",
    "I32", "I64", "F32", "F64", "BF16", "SUM", "MAX", "MIN", "PROD", "BAND", "BOR", "BXOR", "LAND",
    "LOR", "CFG_NO_MODEL", "CFG_STATIC_TILES", "CFG_HIST_DIRECT", "CFG_HIST_TEAM_COPY", "CFG_HIST_PARTITION", "CFG_HIST_RANGES", "CFG_HIST_TILE_SORT", "CFG_EXACT_THREAD_MAP", "reduce_array", "reduce_array_plan", "reduce_loc", "reduce_multi", "histogram", "generic_power", "region_axpy_sum", "udr_declare", "reduce_udr", "queue_chunk",
    "queue_map", "axpy_sum_queue",
]

_OPS = {"sum": SUM, "max": MAX, "min": MIN, "prod": PROD, "band": BAND, "bor": BOR, "bxor": BXOR,
        "land": LAND, "lor": LOR}


def load():
    """Load the library (raises if it is not built)."""
    return _lib.load()


def version() -> str:
    return load().omprt_version().decode()


def _op(op) -> int:
    return _OPS[op] if isinstance(op, str) else int(op)


def dtype_code(t) -> int:
    import torch
    m = {torch.int32: I32, torch.int64: I64, torch.float32: F32, torch.float64: F64,
         torch.bfloat16: BF16}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def _stream(stream) -> int | None:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _cfg(config):
    if config is None:
        return None
    if isinstance(config, Config):
        return ctypes.byref(config)
    c = Config()
    c.num_teams = config.get("teams", 0)
    c.threads_per_team = config.get("threads", 0)
    c.vec_bytes = config.get("vec", 0)
    c.unroll = config.get("unroll", 0)
    c.tile_kib = config.get("tile_kib", 0)
    c.flags = config.get("flags", 0)
    return ctypes.byref(c)


def _sched(n, teams, threads, dist_chunk=0, chunk=0) -> Sched:
    return Sched(int(n), int(teams), int(threads), int(dist_chunk), int(chunk))


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor required")
    return t.data_ptr() or None


# ---------------------------------------------------------------- schedules

def for_static_bounds(n, teams, threads, dist_chunk, chunk, team, thread, j):
    """(lb, ub, is_last) of the j-th chunk of (team, thread); lb == ub == n past the end."""
    lb, ub, last = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    s = _sched(n, teams, threads, dist_chunk, chunk)
    check(load().omprt_for_static_bounds(ctypes.byref(s), team, thread, j, ctypes.byref(lb),
                                         ctypes.byref(ub), ctypes.byref(last)),
          "for_static_bounds")
    return lb.value, ub.value, last.value


def sched_count(n, teams, threads, dist_chunk, chunk, team, thread):
    """(n_chunks, n_iters) of (team, thread)."""
    c, it = ctypes.c_int64(), ctypes.c_int64()
    s = _sched(n, teams, threads, dist_chunk, chunk)
    check(load().omprt_sched_count(ctypes.byref(s), team, thread, ctypes.byref(c),
                                   ctypes.byref(it)), "sched_count")
    return c.value, it.value


def static_map(n, teams, threads, dist_chunk, chunk, owner, count, stream=None):
    """GPU iteration map into int32 owner[n] / int32-or-uint32 count[n] (count zeroed by caller)."""
    s = _sched(n, teams, threads, dist_chunk, chunk)
    check(load().omprt_static_map(ctypes.byref(s), _ptr(owner), _ptr(count), _stream(stream)),
          "static_map")


def empty_region(n, teams, threads, dist_chunk=0, chunk=0, iters=None, stream=None):
    """Empty target region; iters (int64 device tensor or None) gets += the iteration count."""
    s = _sched(n, teams, threads, dist_chunk, chunk)
    check(load().omprt_empty_region(ctypes.byref(s), _ptr(iters), _stream(stream)),
          "empty_region")


# ---------------------------------------------------------------- reductions

def reduce(inp, op, x, config=None, stream=None, n=None):
    """x <- x (op) fold(op, inp[:n]) on the GPU (inp 1-D contiguous, x one element)."""
    if not inp.is_contiguous():
        raise ValueError("input must be contiguous")
    nn = inp.numel() if n is None else int(n)
    check(load().omprt_reduce(_ptr(inp) if nn else (inp.data_ptr() or None), nn, dtype_code(inp),
                              _op(op), _ptr(x), _cfg(config), _stream(stream)), "reduce")


def reduce_noalloc(inp, op, x, config=None, stream=None, n=None):
    """reduce() through the entry point that allocates nothing (cross-team state in a
    fixed device array; at most 4096 teams; calls on one device must not overlap)."""
    if not inp.is_contiguous():
        raise ValueError("input must be contiguous")
    nn = inp.numel() if n is None else int(n)
    check(load().omprt_reduce_noalloc(_ptr(inp) if nn else (inp.data_ptr() or None), nn,
                                      dtype_code(inp), _op(op), _ptr(x), _cfg(config),
                                      _stream(stream)), "reduce_noalloc")


def histogram(keys, bins, hist, config=None, stream=None):
    """hist[k] += number of keys equal to k, for k in [0, bins) (int32 keys and hist)."""
    if not keys.is_contiguous():
        raise ValueError("keys must be contiguous")
    if hist.numel() < bins:
        raise ValueError("hist has fewer than bins entries")
    n = keys.numel()
    check(load().omprt_histogram(_ptr(keys) if n else None, n, int(bins), _ptr(hist), _cfg(config),
                                 _stream(stream)), "histogram")


def generic_power(diag, v, iters, lam, teams=0, threads=0, stream=None):
    """Generic-mode power iteration on diag(diag): iters times w = diag * v,
    v = w / |w|; lam[0] <- |w| of the last step.  v (fp32, contiguous) is
    updated in place; one kernel launch.  teams 1: one team; T > 1: T
    co-resident teams; 0: chosen from n."""
    if not diag.is_contiguous() or not v.is_contiguous():
        raise ValueError("diag and v must be contiguous")
    if diag.numel() != v.numel():
        raise ValueError("diag and v differ in length")
    if dtype_code(diag) != F32 or dtype_code(v) != F32 or dtype_code(lam) != F32:
        raise ValueError("diag, v and lam must be float32")
    check(load().omprt_generic_power(_ptr(diag), _ptr(v), v.numel(), int(iters), int(teams),
                                     int(threads), _ptr(lam), _stream(stream)), "generic_power")


def udr_declare(type_def, initializer, combiner, body, acc_bytes, dtype):
    """declare reduction: compile the user's reduction type (named omp_type), initializer
    (sets omp_priv), combiner (folds omp_in into omp_out) and loop body (folds omp_elem at
    position omp_i into omp_priv) for inputs of `dtype` (a dtype code); returns a handle."""
    src = _lib.UdrSource(type_def.encode(), initializer.encode(), combiner.encode(),
                         body.encode(), int(acc_bytes))
    h = ctypes.c_int32(-1)
    check(load().omprt_udr_declare(ctypes.byref(src), int(dtype), ctypes.byref(h)), "udr_declare")
    return h.value


def reduce_udr(handle, inp, x, config=None, stream=None):
    """x <- combiner(x, reduction of inp) under a declared reduction; x is a device
    tensor holding one omp_type (its bytes)."""
    if not inp.is_contiguous():
        raise ValueError("input must be contiguous")
    n = inp.numel()
    check(load().omprt_reduce_udr(int(handle), _ptr(inp) if n else None, n, _ptr(x), _cfg(config),
                                  _stream(stream)), "reduce_udr")


def reduce_multi(inp, variables, config=None, stream=None):
    """Several reduction variables over the same input in one pass:
    variables = [(op, x tensor), ...] with distinct ops among sum / max / min."""
    if not inp.is_contiguous():
        raise ValueError("input must be contiguous")
    n = inp.numel()
    ops = (ctypes.c_int32 * len(variables))(*[_op(op) for op, _ in variables])
    xs = (ctypes.c_void_p * len(variables))(*[_ptr(x) for _, x in variables])
    check(load().omprt_reduce_multi(_ptr(inp) if n else None, n, dtype_code(inp), len(variables),
                                    ops, xs, _cfg(config), _stream(stream)), "reduce_multi")


def reduce_loc(inp, op, val, idx, config=None, stream=None):
    """maxloc ("max") / minloc ("min"): (val[0], idx[0]) <- the first (value, position)
    pair by value then smaller position over (val[0], idx[0]) and (inp[i], i)."""
    if not inp.is_contiguous():
        raise ValueError("input must be contiguous")
    n = inp.numel()
    check(load().omprt_reduce_loc(_ptr(inp) if n else None, n, dtype_code(inp), _op(op), _ptr(val),
                                  _ptr(idx), _cfg(config), _stream(stream)), "reduce_loc")


def reduce_array(inp, rows, m, op, x, config=None, stream=None):
    """x[j] <- x[j] (op) fold(op, inp[i*m + j] for i < rows), j < m (inp row-major)."""
    if not inp.is_contiguous() or not x.is_contiguous():
        raise ValueError("input and x must be contiguous")
    rows, m = int(rows), int(m)
    if rows * m > inp.numel() or m > x.numel():
        raise ValueError("input or x is smaller than rows x m")
    nz = rows > 0 and m > 0
    check(load().omprt_reduce_array(_ptr(inp) if nz else None, rows, m, dtype_code(inp), _op(op),
                                    _ptr(x) if nz else None, _cfg(config), _stream(stream)),
          "reduce_array")


def reduce_array_plan(rows, m, dtype, op, aligned16=True, config=None):
    """(W, R, col_tiles, row_teams, groups, bytes_per_load, threads, unroll) of a launch."""
    out = (ctypes.c_int64 * 8)()
    check(load().omprt_reduce_array_plan(int(rows), int(m), int(dtype), _op(op), int(aligned16),
                                         _cfg(config), out), "reduce_array_plan")
    return tuple(int(v) for v in out)


def make_segments(items):
    """ctypes Segment array from [(input tensor, op, x tensor[, n]), ...]."""
    arr = (Segment * len(items))()
    for i, it in enumerate(items):
        inp, op, x = it[0], it[1], it[2]
        n = it[3] if len(it) > 3 else inp.numel()
        arr[i] = Segment(inp.data_ptr() or None, int(n), dtype_code(inp), _op(op), x.data_ptr())
    return arr


def reduce_batched(segments, config=None, stream=None):
    """All segments in one persistent, graph-replayed launch (see make_segments)."""
    arr = segments if isinstance(segments, ctypes.Array) else make_segments(segments)
    check(load().omprt_reduce_batched(arr, len(arr), _cfg(config), _stream(stream)),
          "reduce_batched")


def reduce_each(segments, config=None, stream=None):
    """The same segments as one plain launch each."""
    arr = segments if isinstance(segments, ctypes.Array) else make_segments(segments)
    check(load().omprt_reduce_each(arr, len(arr), _cfg(config), _stream(stream)), "reduce_each")


def axpy_sum(a, x, y, s, teams=0, threads=0, dist_chunk=0, chunk=0, config=None, stream=None):
    """y <- fmaf(a, x, y) under the exact static schedule; s[0] += sum(updated y)."""
    sch = _sched(x.numel(), teams, threads, dist_chunk, chunk)
    check(load().omprt_axpy_sum(ctypes.c_float(a), _ptr(x) if x.numel() else None,
                                _ptr(y) if y.numel() else None, _ptr(s), ctypes.byref(sch),
                                _cfg(config), _stream(stream)), "axpy_sum")


def region_axpy_sum(a, x, y, s, teams=0, threads=0, dist_chunk=0, chunk=0, chunk2=None,
                    nowait=False, config=None, stream=None):
    """Two loops in one region: y <- fmaf(a, x, y) under schedule(static, chunk) [nowait],
    then s[0] += sum(y) under schedule(static, chunk2) (default: chunk)."""
    sch = _sched(x.numel(), teams, threads, dist_chunk, chunk)
    c2 = chunk if chunk2 is None else chunk2
    check(load().omprt_region_axpy_sum(ctypes.c_float(a), _ptr(x) if x.numel() else None,
                                       _ptr(y) if y.numel() else None, _ptr(s), ctypes.byref(sch),
                                       int(c2), 1 if nowait else 0, _cfg(config), _stream(stream)),
          "region_axpy_sum")


# ---------------------------------------------------------------- dynamic / guided

SCHED_KINDS = {"dynamic": 1, "guided": 2}


def queue_chunk(kind, m, threads, chunk, j):
    """The j-th chunk [lo, hi) of a block of m iterations under schedule(kind, chunk)."""
    lb, ub = ctypes.c_int64(), ctypes.c_int64()
    check(load().omprt_queue_chunk(SCHED_KINDS[kind], int(m), int(threads), int(chunk), int(j),
                                   ctypes.byref(lb), ctypes.byref(ub)), "queue_chunk")
    return lb.value, ub.value


def queue_map(kind, n, teams, threads, dist_chunk, chunk, owner, count, start, tickets=1,
              stream=None):
    """Iteration map under a dynamic / guided schedule (owner, count, chunk start)."""
    sch = _sched(n, teams, threads, dist_chunk, chunk)
    check(load().omprt_queue_map(ctypes.byref(sch), SCHED_KINDS[kind], int(tickets), _ptr(owner),
                                 _ptr(count), _ptr(start), _stream(stream)), "queue_map")


def axpy_sum_queue(kind, a, x, y, s, teams=0, threads=0, dist_chunk=0, chunk=0, stream=None):
    """y <- fmaf(a, x, y) under a dynamic / guided schedule; s[0] += sum(updated y)."""
    sch = _sched(x.numel(), teams, threads, dist_chunk, chunk)
    check(load().omprt_axpy_sum_queue(ctypes.c_float(a), _ptr(x) if x.numel() else None,
                                      _ptr(y) if y.numel() else None, _ptr(s), ctypes.byref(sch),
                                      SCHED_KINDS[kind], _stream(stream)), "axpy_sum_queue")


# ---------------------------------------------------------------- device atomics

_ATOMICS = {"add": ATOMIC_ADD, "inc": ATOMIC_INC, "max": ATOMIC_MAX, "exchange": ATOMIC_EXCHANGE,
            "cas": ATOMIC_CAS}


def atomic_apply(op, target, index, e, old, d=None, stream=None):
    """old[i] <- atomic op on target[index[i]] with operand e[i] (and d[i] for cas);
    all uint32 (torch.int32 storage), one GPU thread per operation."""
    code = _ATOMICS[op] if isinstance(op, str) else int(op)
    check(load().omprt_atomic_apply(code, _ptr(target), target.numel(), _ptr(index), _ptr(e),
                                    _ptr(d), _ptr(old), index.numel(), _stream(stream)),
          "atomic_apply")


# ---------------------------------------------------------------- learned picker

def mlp_param_count(F, H1, H2, K) -> int:
    d = MlpDims(F, H1, H2, K)
    return int(load().omprt_mlp_param_count(ctypes.byref(d)))


def mlp_forward(dims, params, X, Z, stream=None):
    d = MlpDims(*dims)
    check(load().omprt_mlp_forward(ctypes.byref(d), _ptr(params), _ptr(X), X.shape[0], _ptr(Z),
                                   _stream(stream)), "mlp_forward")


def mlp_loss_grad(dims, params, X, y, loss, grads, stream=None):
    d = MlpDims(*dims)
    check(load().omprt_mlp_loss_grad(ctypes.byref(d), _ptr(params), _ptr(X), _ptr(y), X.shape[0],
                                     _ptr(loss), _ptr(grads), _stream(stream)), "mlp_loss_grad")


def mlp_adam(params, m, v, grads, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(load().omprt_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grads), params.numel(),
                                int(step), lr, beta1, beta2, eps, _stream(stream)), "mlp_adam")


def mlp_adam_counted(params, m, v, grads, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                     stream=None):
    """Adam with the step count in the int32 device tensor `step` (advanced by one)."""
    check(load().omprt_mlp_adam_counted(_ptr(params), _ptr(m), _ptr(v), _ptr(grads),
                                        params.numel(), _ptr(step), lr, beta1, beta2, eps,
                                        _stream(stream)), "mlp_adam_counted")


def model_load(path):
    """Load (path) or unload (None) the learned configuration picker."""
    check(load().omprt_model_load(None if path is None else str(path).encode()), "model_load")


def model_features(n, dtype, op, body=0, chunk=-1):
    f = (ctypes.c_float * 16)()
    check(load().omprt_model_features(int(n), int(dtype), _op(op), int(body), int(chunk), f),
          "model_features")
    return list(f)


def resolve_config(n, dtype, op, body=0, chunk=-1, config=None):
    """(dict(teams, threads, vec, unroll), source) with source 0 explicit, 1 model, 2 tuned, 3 heuristic."""
    out = Config()
    src = ctypes.c_int32()
    check(load().omprt_resolve_config(int(n), int(dtype), _op(op), int(body), int(chunk),
                                      _cfg(config), ctypes.byref(out), ctypes.byref(src)),
          "resolve_config")
    return ({"teams": out.num_teams, "threads": out.threads_per_team, "vec": out.vec_bytes,
             "unroll": out.unroll}, src.value)


def tune_set(dtype, op, body, log2n, config):
    check(load().omprt_tune_set(int(dtype), _op(op), int(body), int(log2n), _cfg(config)),
          "tune_set")


# ---------------------------------------------------------------- runtime

def workspace_reserve(max_teams, max_counters=0, stream=None):
    check(load().omprt_workspace_reserve(_stream(stream), int(max_teams), int(max_counters)),
          "workspace_reserve")


def workspace_reset(stream=None):
    check(load().omprt_workspace_reset(_stream(stream)), "workspace_reset")


def workspace_status(stream=None) -> int:
    """Synchronise the stream; 0 when healthy, else the status bits (1 a cross-team wait
    expired, 2 an atomic index out of range, 4 a histogram key out of range, 8 a
    team-shared allocation found no room, 16 an empty region's schedule inconsistent)."""
    v = ctypes.c_int32()
    check(load().omprt_workspace_status(_stream(stream), ctypes.byref(v)), "workspace_status")
    return v.value


def finalize():
    check(load().omprt_finalize(), "finalize")
