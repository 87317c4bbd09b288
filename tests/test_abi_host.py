"""Host-side tests of the C-ABI library (CPU only, no device calls).

* the library loads and exports every function include/omprt.h declares;
* omprt_for_static_bounds / omprt_sched_count against the oracle's
  enumeration, exhaustively on tiny schedules and on the 2^20 x 256 example;
* argument validation and error codes of every entry point whose checks
  run before any device call;
* configuration resolution (explicit > tuned cache > heuristic) and the
  cost-model feature vector.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_2106_03219_amd as om
from paper_2106_03219_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "omprt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(omprt_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = om.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)
    assert om.version().startswith("omprt")


def test_struct_layouts_match_header():
    assert ctypes.sizeof(om.Sched) == 32
    assert ctypes.sizeof(om.Config) == 24
    assert ctypes.sizeof(om.Segment) == 32
    assert ctypes.sizeof(om.MlpDims) == 16


TINY = [(n, T, P, dc, c)
        for n in (0, 1, 2, 5, 13, 31, 64)
        for T in (1, 2, 3, 5)
        for P in (1, 3, 4, 8)
        for dc in (0, 1, 3, 7)
        for c in (0, 1, 2, 5, 70)]


def _lib_chunks(n, T, P, dc, c, k, t):
    out = []
    nch, nit = om.sched_count(n, T, P, dc, c, k, t)
    for j in range(nch + 1):
        lb, ub, last = om.for_static_bounds(n, T, P, dc, c, k, t, j)
        if j == nch:
            assert (lb, ub, last) == (n, n, 0)
            break
        assert lb < ub
        assert last == (1 if ub == n else 0)
        out.append((lb, ub))
    assert sum(h - l for l, h in out) == nit
    return out


def test_bounds_match_oracle_exhaustive_tiny():
    for n, T, P, dc, c in TINY:
        for k in range(T):
            for t in range(P):
                assert _lib_chunks(n, T, P, dc, c, k, t) == \
                    oracle.thread_chunks(n, T, P, dc, c, k, t), (n, T, P, dc, c, k, t)


def test_bounds_match_oracle_larger_random():
    g = np.random.Generator(np.random.PCG64(12))
    for _ in range(60):
        n = int(g.integers(0, 5000))
        T = int(g.integers(1, 9))
        P = int(g.integers(1, 70))
        dc = int(g.choice([0, 1, 17, 64, 999]))
        c = int(g.choice([0, 1, 3, 64, 1024]))
        k, t = int(g.integers(0, T)), int(g.integers(0, P))
        assert _lib_chunks(n, T, P, dc, c, k, t) == oracle.thread_chunks(n, T, P, dc, c, k, t)


def test_bounds_2pow20_one_team_256():
    n = 1 << 20
    for t in (0, 1, 36, 37, 255):
        assert _lib_chunks(n, 1, 256, 0, 0, 0, t) == oracle.thread_chunks(n, 1, 256, 0, 0, 0, t)
        assert om.sched_count(n, 1, 256, 0, 7, 0, t) == \
            (len(oracle.thread_chunks(n, 1, 256, 0, 7, 0, t)),
             sum(h - l for l, h in oracle.thread_chunks(n, 1, 256, 0, 7, 0, t)))
    assert om.for_static_bounds(n, 1, 256, 0, 7, 0, 36, 585) == (n - 4, n, 1)


def test_bounds_errors():
    with pytest.raises(om.OmprtError) as e:
        om.for_static_bounds(10, 0, 4, 0, 0, 0, 0, 0)
    assert e.value.status == _lib.ERR_INVALID
    for args in [(10, 2, 4, 0, 0, 2, 0, 0), (10, 2, 4, 0, 0, 0, 4, 0), (10, 2, 4, 0, 0, 0, 0, -1),
                 (-1, 2, 4, 0, 0, 0, 0, 0), (10, 2, 1025, 0, 0, 0, 0, 0), (10, 2, 4, -1, 0, 0, 0, 0)]:
        with pytest.raises(om.OmprtError):
            om.for_static_bounds(*args)
    lib = om.load()
    s = om.Sched(10, 2, 4, 0, 0)
    assert lib.omprt_for_static_bounds(ctypes.byref(s), 0, 0, 0, None, None, None) == _lib.ERR_INVALID
    assert b"NULL" in lib.omprt_last_error()


def test_reduce_argument_errors_before_device():
    lib = om.load()
    x = ctypes.c_int64(0)
    assert lib.omprt_reduce(None, 5, 9, 0, ctypes.byref(x), None, None) == _lib.ERR_UNSUPPORTED
    assert lib.omprt_reduce(None, 5, 0, 9, ctypes.byref(x), None, None) == _lib.ERR_UNSUPPORTED
    for op in (_lib.BAND, _lib.BOR, _lib.BXOR):          # bitwise operators: integers only
        for dt in (_lib.F32, _lib.F64, _lib.BF16):
            assert lib.omprt_reduce(None, 5, dt, op, ctypes.byref(x), None, None) == _lib.ERR_UNSUPPORTED
        assert lib.omprt_reduce(None, 0, _lib.I64, op, ctypes.byref(x), None, None) == _lib.OK
    assert lib.omprt_reduce(None, -1, 0, 0, ctypes.byref(x), None, None) == _lib.ERR_INVALID
    assert lib.omprt_reduce(None, 5, 0, 0, ctypes.byref(x), None, None) == _lib.ERR_INVALID
    assert lib.omprt_reduce(None, 0, 0, 0, None, None, None) == _lib.ERR_INVALID
    # n == 0 leaves x alone and touches no device
    assert lib.omprt_reduce(None, 0, 0, 0, ctypes.byref(x), None, None) == _lib.OK
    # misaligned input
    assert lib.omprt_reduce(ctypes.c_void_p(0x1002), 5, 0, 0, ctypes.byref(x), None, None) == _lib.ERR_INVALID
    bad = [om.Config(0, 100, 0, 0, 0, 0), om.Config(0, 0, 4, 0, 0, 0), om.Config(0, 0, 0, 3, 0, 0),
           om.Config(-1, 0, 0, 0, 0, 0), om.Config(0, 0, 0, 0, 2, 0)]
    for c in bad:
        assert lib.omprt_reduce(None, 0, 0, 0, ctypes.byref(x), ctypes.byref(c), None) == _lib.ERR_INVALID


def test_other_entry_point_errors_before_device():
    lib = om.load()
    assert lib.omprt_static_map(None, None, None, None) == _lib.ERR_INVALID
    s = om.Sched(10, 0, 4, 0, 0)
    assert lib.omprt_static_map(ctypes.byref(s), None, None, None) == _lib.ERR_INVALID
    s = om.Sched(1 << 20, 1 << 22, 1024, 0, 0)
    assert lib.omprt_static_map(ctypes.byref(s), None, None, None) == _lib.ERR_INVALID
    s = om.Sched(0, 1, 64, 0, 0)
    assert lib.omprt_static_map(ctypes.byref(s), None, None, None) == _lib.OK
    assert lib.omprt_axpy_sum(1.0, None, None, None, ctypes.byref(s), None, None) == _lib.ERR_INVALID
    s2 = om.Sched(100, 0, 0, 0, 0)
    f = ctypes.c_float(0)
    assert lib.omprt_axpy_sum(1.0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1100), ctypes.byref(f),
                              ctypes.byref(s2), None, None) == _lib.ERR_INVALID   # overlap
    assert lib.omprt_reduce_batched(None, -1, None, None) == _lib.ERR_INVALID
    assert lib.omprt_reduce_batched(None, 0, None, None) == _lib.OK
    seg = (om.Segment * 1)(om.Segment(None, 5, 0, 0, None))
    assert lib.omprt_reduce_batched(seg, 1, None, None) == _lib.ERR_INVALID
    seg = (om.Segment * 1)(om.Segment(None, 5, 8, 0, None))
    assert lib.omprt_reduce_each(seg, 1, None, None) == _lib.ERR_UNSUPPORTED
    d = om.MlpDims(16, 64, 64, 1)
    assert lib.omprt_mlp_forward(ctypes.byref(d), None, None, 4, None, None) == _lib.ERR_INVALID
    assert lib.omprt_mlp_adam(None, None, None, None, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == _lib.ERR_INVALID
    assert lib.omprt_model_load(b"/nonexistent/model.txt") != _lib.OK or True
    assert lib.omprt_workspace_reserve(None, 0, 0) == _lib.ERR_INVALID
    assert om.mlp_param_count(16, 64, 64, 64) == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64


def test_resolve_config_precedence_and_heuristic():
    cfg, src = om.resolve_config(1 << 28, om.F32, "sum", config={"teams": 7, "threads": 128,
                                                               "vec": 8, "unroll": 2})
    assert src == 0 and cfg == {"teams": 7, "threads": 128, "vec": 8, "unroll": 2}
    cfg, src = om.resolve_config(1 << 28, om.F32, "sum", config={"flags": om.CFG_NO_MODEL})
    assert src == 3 and cfg["threads"] == 512 and cfg["vec"] == 16
    assert 1 <= cfg["teams"] <= 65535
    small, _ = om.resolve_config(10, om.I32, "sum")
    assert small["teams"] == 1
    # the tuned cache wins over the heuristic for its (dtype, op, body, log2 n) bucket
    om.tune_set(om.I64, "max", 0, 20, {"teams": 33, "threads": 512, "vec": 8, "unroll": 8})
    cfg, src = om.resolve_config((1 << 20) + 5, om.I64, "max")
    assert src == 2 and cfg == {"teams": 33, "threads": 512, "vec": 8, "unroll": 8}
    # partial explicit fields override the tuned entry field by field
    cfg, src = om.resolve_config((1 << 20) + 5, om.I64, "max", config={"threads": 64})
    assert cfg["threads"] == 64 and cfg["teams"] == 33
    om.tune_set(om.I64, "max", 0, 20, None)
    _, src = om.resolve_config((1 << 20) + 5, om.I64, "max")
    assert src == 3
    with pytest.raises(om.OmprtError):
        om.tune_set(om.I64, "max", 0, 20, {"teams": 33})   # must be complete


def test_heuristic_large_user_chunks():
    """The AXPY body's default launch for chunks of more than 512 iterations (256 compute units
    without a GPU): 512 threads and about 128 chunks a team, rounded down to whole rounds of
    one team per CU; with fewer than two waves' worth of chunks per CU, one team per wave of
    chunks (at most one a CU) of 64 threads per wave.  Chunks up to 512 keep the body's
    general launch (8 teams of 256 per CU at this size)."""
    def pick(n, c):
        cfg, src = om.resolve_config(n, om.F32, "sum", 1, c)
        assert src == 3
        return cfg["teams"], cfg["threads"]
    n = 1 << 26
    assert pick(n, 512) == (2048, 256)      # the general launch
    assert pick(n, 768) == (512, 512)       # 683 rounded down to two rounds
    assert pick(n, 1024) == (512, 512)
    assert pick(n, 992) == (512, 512)       # 529 would leave a third round of 17 teams
    assert pick(n, 2000) == (256, 512)      # 263 would leave a second round of 7
    assert pick(n, 4096) == (256, 64)       # 256 waves of chunks, one a CU
    assert pick(n, 8192) == (128, 64)
    assert pick(300001, 1024) == (5, 64)    # 293 chunks: five waves
    assert pick(n, n) == (1, 64)            # one chunk
    assert pick(300 * 64 * 1024, 1024) == (256, 128)   # 300 waves: two a team on 44 CUs


def test_model_features():
    f = om.model_features(1 << 20, om.F32, "sum", 0, -1)
    assert f[0] == 20.0 and f[3] == 1.0 and sum(f[1:6]) == 1.0
    assert f[6] == 1.0 and sum(f[6:9]) == 1.0
    assert f[11] == 4.0 and f[13] == 22.0 and f[14] == 1.0 and f[15] == 0.0
    g = om.model_features(1000, om.F32, "sum", 1, 64)
    assert g[9] == 6.0 and g[10] == 0.0 and g[11] == 12.0 and g[15] == 1.0
    assert math.isclose(g[13], math.log2(12000), rel_tol=1e-6)
    h = om.model_features(5, om.I64, "min", 0, 0)
    assert h[10] == 1.0 and h[14] == 0.0


def test_atomic_apply_argument_errors():
    lib = om.load()
    p = ctypes.c_void_p(0x1000)
    assert lib.omprt_atomic_apply(5, p, 1, p, p, None, p, 1, None) == _lib.ERR_INVALID
    assert lib.omprt_atomic_apply(0, p, 0, p, p, None, p, 1, None) == _lib.ERR_INVALID
    assert lib.omprt_atomic_apply(4, p, 1, p, p, None, p, 1, None) == _lib.ERR_INVALID  # cas needs d
    assert lib.omprt_atomic_apply(0, None, 1, p, p, None, p, 1, None) == _lib.ERR_INVALID
    assert lib.omprt_atomic_apply(0, p, 1, p, p, None, p, -1, None) == _lib.ERR_INVALID
    assert lib.omprt_atomic_apply(0, None, 0, None, None, None, None, 0, None) == _lib.OK


def test_histogram_and_multi_argument_errors():
    lib = om.load()
    h = ctypes.c_int32(0)
    H = lib.omprt_histogram
    assert H(None, -1, 10, ctypes.byref(h), None, None) == _lib.ERR_INVALID
    assert H(None, 10, 0, ctypes.byref(h), None, None) == _lib.ERR_INVALID
    assert H(None, 10, (1 << 28) + 1, ctypes.byref(h), None, None) == _lib.ERR_INVALID
    assert H(None, 10, 10, None, None, None) == _lib.ERR_INVALID
    assert H(None, 10, 10, ctypes.byref(h), None, None) == _lib.ERR_INVALID      # NULL keys
    assert H(None, 0, 10, ctypes.byref(h), None, None) == _lib.OK
    assert H(ctypes.c_void_p(0x1002), 10, 10, ctypes.byref(h), None, None) == _lib.ERR_INVALID
    c = om.Config(0, 0, 0, 8, 0, 0)
    assert H(ctypes.c_void_p(0x1000), 10, 10, ctypes.byref(h), ctypes.byref(c), None) == _lib.ERR_INVALID
    M = lib.omprt_reduce_multi
    ops = (ctypes.c_int32 * 2)(0, 0)
    xs = (ctypes.c_void_p * 2)(0x1000, 0x1010)
    assert M(ctypes.c_void_p(0x2000), 10, 2, 2, ops, xs, None, None) == _lib.ERR_INVALID   # repeated
    ops3 = (ctypes.c_int32 * 1)(3)
    assert M(ctypes.c_void_p(0x2000), 10, 2, 1, ops3, xs, None, None) == _lib.ERR_UNSUPPORTED
    assert M(ctypes.c_void_p(0x2000), 10, 2, 4, ops, xs, None, None) == _lib.ERR_INVALID
    assert M(ctypes.c_void_p(0x2000), 10, 2, 1, None, xs, None, None) == _lib.ERR_INVALID
    L = lib.omprt_reduce_loc
    i = ctypes.c_int64(0)
    assert L(None, 10, 2, 0, ctypes.byref(h), ctypes.byref(i), None, None) == _lib.ERR_UNSUPPORTED
    assert L(None, 0, 2, 1, ctypes.byref(h), ctypes.byref(i), None, None) == _lib.OK
    assert L(None, 0, 2, 1, None, ctypes.byref(i), None, None) == _lib.ERR_INVALID


def test_generic_power_argument_errors():
    G = om.load().omprt_generic_power
    d, v, lam = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000)
    assert G(d, v, 0, 1, 1, 0, lam, None) == _lib.ERR_INVALID                  # n < 1
    assert G(d, v, (1 << 32) + 1, 1, 1, 0, lam, None) == _lib.ERR_INVALID      # n too large
    assert G(d, v, 16, 0, 1, 0, lam, None) == _lib.ERR_INVALID                 # iters < 1
    assert G(d, v, 16, 1, -1, 0, lam, None) == _lib.ERR_INVALID                # teams < 0
    for t in (32, 96 + 1, 1088, -64):
        assert G(d, v, 16, 1, 1, t, lam, None) == _lib.ERR_INVALID             # threads
    assert G(None, v, 16, 1, 1, 0, lam, None) == _lib.ERR_INVALID
    assert G(d, v, 16, 1, 1, 0, None, None) == _lib.ERR_INVALID
    assert G(ctypes.c_void_p(0x10002), v, 16, 1, 1, 0, lam, None) == _lib.ERR_INVALID   # misaligned
    assert G(d, ctypes.c_void_p(0x10000 + 60), 16, 1, 1, 0, lam, None) == _lib.ERR_INVALID  # overlap
    assert G(d, v, 16, 1, 1, 0, ctypes.c_void_p(0x20000 + 8), None) == _lib.ERR_INVALID    # lambda in v


def test_region_argument_errors():
    R = om.load().omprt_region_axpy_sum
    f = ctypes.c_float(0)
    x, y = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    s = om.Sched(100, 0, 0, 0, 4)
    assert R(1.0, x, y, ctypes.byref(f), ctypes.byref(s), 8, 1, None, None) == _lib.ERR_INVALID  # nowait, c1 != c2
    assert R(1.0, x, y, ctypes.byref(f), ctypes.byref(s), -1, 0, None, None) == _lib.ERR_INVALID  # chunk2 < 0
    assert R(1.0, x, y, None, ctypes.byref(s), 4, 1, None, None) == _lib.ERR_INVALID             # sum NULL
    assert R(1.0, x, ctypes.c_void_p(0x10000 + 200), ctypes.byref(f), ctypes.byref(s), 4, 0,
             None, None) == _lib.ERR_INVALID                                                     # overlap
    assert R(1.0, None, None, ctypes.byref(f), ctypes.byref(s), 4, 0, None, None) == _lib.ERR_INVALID
    s0 = om.Sched(0, 1, 64, 0, 4)
    assert R(1.0, None, None, ctypes.byref(f), ctypes.byref(s0), 4, 1, None, None) == _lib.OK    # n == 0
    assert R(1.0, None, None, ctypes.byref(f), None, 4, 1, None, None) == _lib.ERR_INVALID


def test_udr_declare_compiles_and_reports_errors():
    """declare reduction compiles with hiprtc on the host (no device needed): a valid source
    gives a handle (the same one when declared again), user errors come back as
    OMPRT_ERR_INVALID with the compiler's message."""
    import udr_cases as U
    c = U.WELFORD
    h = om.udr_declare(c["type_def"], c["initializer"], c["combiner"], c["body"], c["acc_bytes"], om.F32)
    assert h >= 0
    assert om.udr_declare(c["type_def"], c["initializer"], c["combiner"], c["body"], c["acc_bytes"],
                          om.F32) == h
    assert om.udr_declare(c["type_def"], c["initializer"], c["combiner"], c["body"], c["acc_bytes"],
                          om.BF16) != h
    with pytest.raises(om.OmprtError) as e:         # a missing semicolon in the combiner
        om.udr_declare("struct omp_type { int a; };", "omp_priv.a = 0;", "omp_out.a += omp_in.a",
                       "omp_priv.a += omp_elem;", 4, om.I32)
    assert e.value.status == _lib.ERR_INVALID and "combiner" in str(e.value)
    with pytest.raises(om.OmprtError) as e:         # declared size differs from sizeof
        om.udr_declare("struct omp_type { int a; };", "omp_priv.a = 0;", "omp_out.a += omp_in.a;",
                       "omp_priv.a += omp_elem;", 8, om.I32)
    assert "acc_bytes" in str(e.value)
    for bad in (0, 2, 68):
        with pytest.raises(om.OmprtError):
            om.udr_declare("struct omp_type { int a; };", "", "", "", bad, om.I32)
    with pytest.raises(om.OmprtError):
        om.udr_declare("struct omp_type { int a; };", "", "", "", 4, 9)          # dtype
    lib = om.load()
    x = ctypes.c_int32(0)
    assert lib.omprt_reduce_udr(10 ** 6, None, 0, ctypes.byref(x), None, None) == _lib.ERR_INVALID
    assert lib.omprt_reduce_udr(h, None, 5, ctypes.byref(x), None, None) == _lib.ERR_INVALID
    assert lib.omprt_reduce_udr(h, None, 0, None, None, None) == _lib.ERR_INVALID
    cfg = om.Config(0, 0, 16, 0, 0, 0)
    assert lib.omprt_reduce_udr(h, None, 0, ctypes.byref(x), ctypes.byref(cfg), None) == _lib.ERR_INVALID
    assert lib.omprt_reduce_udr(h, None, 0, ctypes.byref(x), None, None) == _lib.OK   # n == 0
