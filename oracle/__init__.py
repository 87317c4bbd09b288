"""Serial CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The product library never loads it, and it shares
no code with the HIP path: ``oracle.c`` is plain serial C built with gcc,
and this module only marshals numpy arrays into it.

Functions and the definitions they follow (see ``oracle.c`` for the full
statement of each):

* :func:`bal`, :func:`iteration_map`, :func:`thread_chunks` -- OpenMP
  static ``distribute`` / ``for`` schedules (paper sec. 1: the device runtime
  supplies the routines behind compiler-lowered worksharing loops; sec. 3.1:
  one team is one GPU thread block).
* :func:`reduce_int`, :func:`reduce_fp` -- ``reduction(op:x)`` results for
  the identifiers + * max min & | ^ && ||: integer wrap arithmetic, FP64
  Neumaier sums and FP64 products, fmax/fmin folds, 0/1 logical folds.
* :func:`queue_chunks`, :func:`team_queue` -- dynamic / guided worksharing:
  the chunks each distribute block's queue hands out (owners undefined).
* :func:`histogram` -- reduction(+: hist[0:bins]) with hist[key[i]] += 1.
* :func:`power_iteration` -- diagonal power iteration (the generic-mode
  region's workload), FP64.
* :func:`reduce_loc` -- maxloc / minloc (value and position, ties to the
  smaller position).
* :func:`axpy_sum` -- the AXPY worksharing body with fused fmaf.
* :func:`fold_prefixes`, :func:`axpy_prefix_sums` -- the same sum / max / min
  folds and AXPY sums read out at several prefix lengths of one array in one
  pass (the autotuner's instances are prefixes of shared buffers).
* :func:`udr_fold`, :func:`moments` -- a user-defined reduction (declare
  reduction) by its sequential definition: the private copy starts at the
  initializer, the loop body folds the elements in order, the combiner
  folds the result into the original value; and the count, mean and sum of
  squared deviations of a sample by their definitions (exactly rounded
  sums), against which a variance reduction is checked.
* :func:`atomic_serial` -- the five device atomics (sec. 3.1) applied in
  index order.
* :func:`mlp_loss_grad`, :func:`adam` -- the learned-configuration
  extension's network in FP64 (not from the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SUM, MAX, MIN, PROD, BAND, BOR, BXOR, LAND, LOR = range(9)
_OPS = {"sum": SUM, "max": MAX, "min": MIN, "prod": PROD, "band": BAND, "bor": BOR,
        "bxor": BXOR, "land": LAND, "lor": LOR}
_FP_DT = {np.dtype(np.float32): 0, np.dtype(np.float64): 1}

_lib = None


def build() -> str:
    """Compile oracle.c with gcc -O2 (no fast-math, single thread)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, p = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.oracle_bal.argtypes = [i64, i64, i64, p, p]
    lib.oracle_bal.restype = None
    lib.oracle_map.argtypes = [i64, i64, i64, i64, i64, p, p]
    lib.oracle_map.restype = ctypes.c_int
    lib.oracle_thread_chunks.argtypes = [i64, i64, i64, i64, i64, i64, i64, p, p, i64]
    lib.oracle_thread_chunks.restype = i64
    lib.oracle_reduce_i32.argtypes = [p, i64, ctypes.c_int, i32]
    lib.oracle_reduce_i32.restype = i32
    lib.oracle_reduce_i64.argtypes = [p, i64, ctypes.c_int, i64]
    lib.oracle_reduce_i64.restype = i64
    lib.oracle_reduce_fp.argtypes = [p, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double, p]
    lib.oracle_reduce_fp.restype = ctypes.c_double
    lib.oracle_axpy_sum.argtypes = [ctypes.c_float, p, p, i64, ctypes.c_double]
    lib.oracle_axpy_sum.restype = ctypes.c_double
    lib.oracle_mlp_loss_grad.argtypes = [p, p, i64, i64, i64, i64, i64] + [p] * 13
    lib.oracle_mlp_loss_grad.restype = ctypes.c_double
    lib.oracle_adam.argtypes = [p, p, p, p, i64, i64] + [ctypes.c_double] * 4
    lib.oracle_adam.restype = None
    lib.oracle_atomic_serial.argtypes = [ctypes.c_int, p, i64, p, p, p, p, i64]
    lib.oracle_atomic_serial.restype = i64
    lib.oracle_power_iteration.argtypes = [p, p, i64, i32, p]
    lib.oracle_power_iteration.restype = None
    lib.oracle_histogram.argtypes = [p, i64, i32, p]
    lib.oracle_histogram.restype = i64
    lib.oracle_reduce_loc.argtypes = [p, i64, ctypes.c_int, ctypes.c_int, i64, ctypes.c_double, i64,
                                      p, p, p]
    lib.oracle_reduce_loc.restype = None
    lib.oracle_queue_chunks.argtypes = [ctypes.c_int, i64, i64, i64, p, p, i64]
    lib.oracle_queue_chunks.restype = i64
    lib.oracle_team_queue.argtypes = [ctypes.c_int, i64, i64, i64, i64, i64, i64, p, p, i64]
    lib.oracle_team_queue.restype = i64
    lib.oracle_fold_prefixes.argtypes = [p, ctypes.c_int, ctypes.c_int, ctypes.c_double, i64, p, i64,
                                         p, p]
    lib.oracle_fold_prefixes.restype = ctypes.c_int
    lib.oracle_axpy_prefix_sums.argtypes = [ctypes.c_float, p, p, ctypes.c_double, p, i64, p]
    lib.oracle_axpy_prefix_sums.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def bal(m: int, p: int, t: int) -> tuple[int, int]:
    """Balanced share [lo, hi) of worker t when m iterations go to p workers."""
    lo, hi = ctypes.c_int64(), ctypes.c_int64()
    _load().oracle_bal(m, p, t, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def iteration_map(n: int, teams: int, threads: int, dist_chunk: int = 0,
                  chunk: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """(owner, count) arrays of the static schedule: owner[i] = team*P+thread."""
    owner = np.full(n, -1, dtype=np.int32)
    count = np.zeros(n, dtype=np.uint32)
    rc = _load().oracle_map(n, teams, threads, dist_chunk, chunk, _ptr(owner), _ptr(count))
    if rc != 0:
        raise ValueError("invalid schedule arguments")
    return owner, count


def thread_chunks(n: int, teams: int, threads: int, dist_chunk: int, chunk: int,
                  team: int, thread: int) -> list[tuple[int, int]]:
    """The non-empty chunks [lo, hi) thread `thread` of team `team` executes, in order."""
    lib = _load()
    cnt = lib.oracle_thread_chunks(n, teams, threads, dist_chunk, chunk, team, thread,
                                   None, None, 0)
    lo = np.zeros(max(cnt, 1), dtype=np.int64)
    hi = np.zeros(max(cnt, 1), dtype=np.int64)
    lib.oracle_thread_chunks(n, teams, threads, dist_chunk, chunk, team, thread,
                             _ptr(lo), _ptr(hi), cnt)
    return [(int(lo[i]), int(hi[i])) for i in range(cnt)]


def reduce_int(a: np.ndarray, op: str, x: int = 0) -> int:
    """x (op) fold(op, a) for int32/int64 arrays, with two's-complement wrap."""
    a = np.ascontiguousarray(a)
    lib = _load()
    if a.dtype == np.int32:
        return int(lib.oracle_reduce_i32(_ptr(a), a.size, _OPS[op], int(np.int32(x))))
    if a.dtype == np.int64:
        return int(lib.oracle_reduce_i64(_ptr(a), a.size, _OPS[op], int(np.int64(x))))
    raise TypeError(a.dtype)


def reduce_fp(a: np.ndarray, op: str, x: float = 0.0, bf16: bool = False,
              want_abs: bool = False):
    """x (op) fold(op, a) in FP64 (Neumaier for sums, fmax/fmin otherwise).

    ``a`` is float32 or float64, or uint16 holding bfloat16 bits when
    ``bf16`` is set.  With ``want_abs`` also returns sum |a_i|.
    """
    a = np.ascontiguousarray(a)
    if bf16:
        if a.dtype != np.uint16:
            raise TypeError("bf16 data must be passed as uint16 bits")
        dt = 2
    else:
        dt = _FP_DT[a.dtype]
    s_abs = ctypes.c_double()
    r = _load().oracle_reduce_fp(_ptr(a), a.size, dt, _OPS[op], float(x),
                                 ctypes.byref(s_abs) if want_abs else None)
    return (r, s_abs.value) if want_abs else r


_PREFIX_DT = {np.dtype(np.int32): 0, np.dtype(np.int64): 1, np.dtype(np.float32): 2,
              np.dtype(np.float64): 3}


def fold_prefixes(a: np.ndarray, op: str, lens, x=None, bf16: bool = False):
    """The sum / max / min fold of a[0..L) for every L in lens, in one pass: a list in
    the order of lens, each what reduce_int / reduce_fp gives for that prefix with
    the same x (default: the op's identity).  Integers as int, floats as float."""
    a = np.ascontiguousarray(a)
    dt = 4 if bf16 else _PREFIX_DT[a.dtype]
    lens = np.asarray(lens, dtype=np.int64)
    order = np.argsort(lens, kind="stable")
    sl = np.ascontiguousarray(lens[order])
    if sl.size and (sl[0] < 0 or sl[-1] > a.size):
        raise ValueError("prefix length outside the array")
    out_i = np.zeros(sl.size, np.int64)
    out_f = np.zeros(sl.size, np.float64)
    if dt <= 1:
        info = np.iinfo(a.dtype)
        xi = 0 if op == "sum" else int(info.min if op == "max" else info.max)
        xi = xi if x is None else int(x)
        xf = 0.0
    else:
        xf = 0.0 if op == "sum" else (-np.inf if op == "max" else np.inf)
        xf = xf if x is None else float(x)
        xi = 0
    if _load().oracle_fold_prefixes(_ptr(a), dt, _OPS[op], xf, xi, _ptr(sl), sl.size,
                                    _ptr(out_i), _ptr(out_f)) != 0:
        raise ValueError("bad op or lengths")
    res = [None] * sl.size
    for k, j in enumerate(order):
        res[j] = int(out_i[k]) if dt <= 1 else float(out_f[k])
    return res


def axpy_prefix_sums(a: float, x: np.ndarray, y: np.ndarray, lens, s_orig: float = 0.0):
    """(y', sums): y' = fmaf(a, x, y) over the longest prefix (a new array), and for
    every L in lens the FP64 sum of y'[0..L) from s_orig, as axpy_sum gives it."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    lens = np.asarray(lens, dtype=np.int64)
    order = np.argsort(lens, kind="stable")
    sl = np.ascontiguousarray(lens[order])
    top = int(sl[-1]) if sl.size else 0
    if top > x.size or top > y.size:
        raise ValueError("prefix length outside the arrays")
    y2 = np.array(y[:top], dtype=np.float32, copy=True)
    out = np.zeros(sl.size, np.float64)
    if _load().oracle_axpy_prefix_sums(ctypes.c_float(a), _ptr(x), _ptr(y2), float(s_orig),
                                       _ptr(sl), sl.size, _ptr(out)) != 0:
        raise ValueError("bad lengths")
    sums = [0.0] * sl.size
    for k, j in enumerate(order):
        sums[j] = float(out[k])
    return y2, sums


def axpy_sum(a: float, x: np.ndarray, y: np.ndarray, s_orig: float = 0.0):
    """Returns (y_new, sum) with y_new[i] = fmaf(a, x[i], y[i]); y is not modified."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y2 = np.array(y, dtype=np.float32, copy=True)
    s = _load().oracle_axpy_sum(ctypes.c_float(a), _ptr(x), _ptr(y2), x.size, float(s_orig))
    return y2, s


def mlp_loss_grad(X, y, params, want_grad=True):
    """Mean softmax-CE loss (and FP64 gradients) of the F->H1->H2->K ReLU MLP.

    ``params`` = dict with W1[H1,F], b1[H1], W2[H2,H1], b2[H2], W3[K,H2], b3[K].
    Returns (loss, logits, grads-dict or None).
    """
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.int32)
    P = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in params.items()}
    B, F = X.shape
    H1, H2, K = P["W1"].shape[0], P["W2"].shape[0], P["W3"].shape[0]
    Z = np.zeros((B, K))
    g = {k: np.zeros_like(v) for k, v in P.items()} if want_grad else None
    gp = [_ptr(g[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3")] if want_grad else [None] * 6
    loss = _load().oracle_mlp_loss_grad(
        _ptr(X), _ptr(y), B, F, H1, H2, K,
        _ptr(P["W1"]), _ptr(P["b1"]), _ptr(P["W2"]), _ptr(P["b2"]),
        _ptr(P["W3"]), _ptr(P["b3"]), _ptr(Z), *gp)
    return loss, Z, g


def adam(w, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One FP64 Adam step at step number t >= 1; returns new (w, m, v)."""
    w = np.array(w, dtype=np.float64, copy=True)
    m = np.array(m, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    g = np.ascontiguousarray(g, dtype=np.float64)
    _load().oracle_adam(_ptr(w), _ptr(m), _ptr(v), _ptr(g), w.size, t, lr, beta1, beta2, eps)
    return w, m, v


ATOMIC_OPS = {"add": 0, "inc": 1, "max": 2, "exchange": 3, "cas": 4}


def atomic_serial(op, target, index, e, d=None):
    """Apply the atomics in index order; returns (new targets, old values, skipped)."""
    t = np.array(target, dtype=np.uint32, copy=True)
    index = np.ascontiguousarray(index, dtype=np.uint32)
    e = np.ascontiguousarray(e, dtype=np.uint32)
    dd = np.ascontiguousarray(d if d is not None else np.zeros_like(e), dtype=np.uint32)
    old = np.zeros(index.size, dtype=np.uint32)
    code = ATOMIC_OPS[op] if isinstance(op, str) else int(op)
    sk = _load().oracle_atomic_serial(code, _ptr(t), t.size, _ptr(index), _ptr(e), _ptr(dd),
                                      _ptr(old), index.size)
    return t, old, int(sk)


def reduce_array(a2d, op, x, bf16=False):
    """reduction(op: x[0:m]) over the rows of a row-major (rows, m) block:
    x[j] (op) fold_i a2d[i, j] for every column j, each column folded exactly as
    reduce_int / reduce_fp fold a 1-D array.  Returns a list of m results."""
    a2d = np.asarray(a2d)
    out = []
    for j in range(a2d.shape[1]):
        col = np.ascontiguousarray(a2d[:, j])
        if col.dtype in (np.int32, np.int64):
            out.append(reduce_int(col, op, x[j]))
        else:
            out.append(reduce_fp(col, op, x[j], bf16=bf16))
    return out


QUEUE_KINDS = {"dynamic": 0, "guided": 1}


def queue_chunks(kind, m, P, c):
    """Chunks [lo, hi) (offsets in a block of m iterations) of schedule(kind, c), in order."""
    lib = _load()
    k = QUEUE_KINDS[kind]
    cnt = lib.oracle_queue_chunks(k, m, P, c, None, None, 0)
    if cnt < 0:
        raise ValueError("invalid schedule arguments")
    lo = np.zeros(max(cnt, 1), dtype=np.int64)
    hi = np.zeros(max(cnt, 1), dtype=np.int64)
    lib.oracle_queue_chunks(k, m, P, c, _ptr(lo), _ptr(hi), cnt)
    return [(int(lo[i]), int(hi[i])) for i in range(cnt)]


def team_queue(kind, n, T, P, dc, c, team):
    """Absolute chunks team `team`'s queues hand out, block by block, in order."""
    lib = _load()
    k = QUEUE_KINDS[kind]
    cnt = lib.oracle_team_queue(k, n, T, P, dc, c, team, None, None, 0)
    if cnt < 0:
        raise ValueError("invalid schedule arguments")
    lo = np.zeros(max(cnt, 1), dtype=np.int64)
    hi = np.zeros(max(cnt, 1), dtype=np.int64)
    lib.oracle_team_queue(k, n, T, P, dc, c, team, _ptr(lo), _ptr(hi), cnt)
    return [(int(lo[i]), int(hi[i])) for i in range(cnt)]


_LOC_DT = {np.dtype(np.int32): 0, np.dtype(np.int64): 1, np.dtype(np.float32): 2,
           np.dtype(np.float64): 3}


def reduce_loc(a, op, x_val, x_idx, bf16=False):
    """(value, position) of maxloc (op "max") / minloc ("min") over (x_val, x_idx)
    and (a[i], i); integers as int, floating values as float."""
    a = np.ascontiguousarray(a)
    dt = 4 if bf16 else _LOC_DT[a.dtype]
    vi, vf, pos = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    integer = dt in (0, 1)
    _load().oracle_reduce_loc(_ptr(a), a.size, dt, _OPS[op], int(x_val) if integer else 0,
                              0.0 if integer else float(x_val), int(x_idx), ctypes.byref(vi),
                              ctypes.byref(vf), ctypes.byref(pos))
    return (vi.value if integer else vf.value), pos.value


def histogram(keys, bins, hist=None):
    """(hist + counts of each key in [0, bins), number of keys outside it); int32 wrap."""
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    h = np.zeros(bins, dtype=np.int32) if hist is None else np.array(hist, dtype=np.int32, copy=True)
    sk = _load().oracle_histogram(_ptr(keys), keys.size, int(bins), _ptr(h))
    return h, int(sk)


def power_iteration(d, v0, iters):
    """(v after iters steps, lambda) of w = d*v; s = sum w^2; v = w / sqrt(s), in FP64."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    v = np.array(v0, dtype=np.float64, copy=True)
    lam = ctypes.c_double()
    _load().oracle_power_iteration(_ptr(d), _ptr(v), d.size, int(iters), ctypes.byref(lam))
    return v, lam.value


# ---------------------------------------------------------------- declare reduction

def udr_fold(values, x0, init, body, combiner):
    """x0 combined with the sequential fold of `values` by a user-defined reduction:
    priv = init(); priv = body(priv, v_i, i) for i = 0, 1, ...; return combiner(x0, priv).
    (OpenMP: the private copy is initialised by the initializer, updated by the loop body,
    and combined into the original list item by the combiner.)"""
    priv = init()
    for i, v in enumerate(values):
        priv = body(priv, v, i)
    return combiner(x0, priv)


def moments(x):
    """(n, mean, M2) of a sample by definition, in FP64 with exactly rounded sums:
    mean = sum(x) / n and M2 = sum((x - mean)^2)."""
    import math
    xs = [float(v) for v in np.asarray(x).ravel()]
    n = len(xs)
    if n == 0:
        return 0.0, 0.0, 0.0
    mean = math.fsum(xs) / n
    return float(n), mean, math.fsum((v - mean) ** 2 for v in xs)
