"""Helpers shared by the GPU parity tests: device inputs, host copies for
the oracle, and the tolerance rules.

FP32/BF16 sums: |got - ref| <= 1e-6 |ref| (ref = FP64 oracle), or, when the
exact sum is 0, |got| <= 1e-6 * sum|x|.  FP64 sums: 1e-12 relative.
Integers, max/min and iteration maps: bit-exact.

Every floating sum checked is also reported: its relative error against the
oracle, rel = |got - ref| / |ref|, and the condition number of the sum,
kappa = sum|x_i| / |sum x_i| (rel / kappa near the unit roundoff means the
error is what the data's cancellation explains).  The records collect in
ERRORS, one per result with the test that made it; the session's summary
prints the worst per test, and OMPRT_ERROR_REPORT=<path> writes them all as
JSON.
"""
from __future__ import annotations

import math
import os

import numpy as np
import torch

import oracle
import synth

TOL_F32 = 1e-6
TOL_F64 = 1e-12
TORCH_DT = {synth.I32: torch.int32, synth.I64: torch.int64, synth.F32: torch.float32,
            synth.F64: torch.float64, synth.BF16: torch.bfloat16}
OPS = ("sum", "max", "min")


def to_device(a: np.ndarray, dtype: int) -> torch.Tensor:
    if dtype == synth.BF16:
        return torch.from_numpy(a.view(np.int16).copy()).cuda().view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t: torch.Tensor) -> np.ndarray:
    if t.dtype == torch.bfloat16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def identity(dtype: int, op: str):
    if op == "sum":
        return 0
    if dtype in (synth.I32, synth.I64):
        info = np.iinfo(np.int32 if dtype == synth.I32 else np.int64)
        return info.min if op == "max" else info.max
    return -np.inf if op == "max" else np.inf


def x_tensor(dtype: int, op: str, value) -> torch.Tensor:
    """One-element x with the library's output type (bf16 sum -> float32)."""
    if dtype == synth.BF16 and op == "sum":
        return torch.tensor([float(value)], dtype=torch.float32, device="cuda")
    return torch.tensor([value], dtype=TORCH_DT[dtype], device="cuda")


def oracle_value(host: np.ndarray, dtype: int, op: str, x0):
    """(value, abs_sum or None) from the oracle."""
    if dtype in (synth.I32, synth.I64):
        return oracle.reduce_int(host, op, int(x0)), None
    if dtype == synth.BF16:
        xv = float(x0) if op == "sum" else float(torch.tensor([x0], dtype=torch.bfloat16).float())
        return oracle.reduce_fp(host, op, xv, bf16=True, want_abs=True)
    return oracle.reduce_fp(host, op, float(x0), want_abs=True)


ERRORS: list[dict] = []
DT_NAME = {synth.I32: "i32", synth.I64: "i64", synth.F32: "f32", synth.F64: "f64",
           synth.BF16: "bf16"}


def sum_error(got: float, ref: float, abs_sum: float | None) -> tuple[float, float]:
    """(rel, kappa) of a floating sum against its oracle value.  With an exact sum of
    0, rel is measured against sum|x| instead and kappa is infinite."""
    got, ref = float(got), float(ref)
    a = float(abs_sum) if abs_sum is not None else abs(ref)
    if ref == 0.0:
        return (abs(got) / a if a > 0 else abs(got)), math.inf
    return abs(got - ref) / abs(ref), a / abs(ref)


def record_error(what: str, dtype: int, rel: float, kappa: float, n: int | None = None):
    ERRORS.append({"test": os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0],
                   "what": what, "dtype": DT_NAME.get(dtype, str(dtype)), "n": n,
                   "rel": rel, "kappa": kappa})


def check_value(got, ref, abs_sum, dtype: int, op: str, what: str = "", n: int | None = None):
    """Assert the result against the oracle's.  Returns (rel, kappa) for a floating
    sum (also recorded in ERRORS), None for exact results."""
    if dtype in (synth.I32, synth.I64) or op != "sum":
        if op != "sum" and dtype not in (synth.I32, synth.I64):
            assert float(got) == float(ref), (what, got, ref)
        else:
            assert int(got) == int(ref), (what, got, ref)
        return None
    tol = TOL_F64 if dtype == synth.F64 else TOL_F32
    rel, kappa = sum_error(got, ref, abs_sum)
    record_error(what, dtype, rel, kappa, n)
    if ref == 0.0:
        assert abs(float(got)) <= tol * abs_sum, (what, got, ref, "rel", rel)
    else:
        assert abs(float(got) - ref) <= tol * abs(ref), (what, got, ref, "rel", rel, "kappa", kappa)
    return rel, kappa


def check_axpy(y_got: np.ndarray, s_got, y_ref: np.ndarray, s_ref: float, s0: float = 0.0,
               what=""):
    """AXPY body with a sum: y bit for bit (one fused rounding on both sides), the sum
    of the updated y within the fp32 tolerance (recorded with its kappa)."""
    assert np.array_equal(np.asarray(y_got).view(np.uint32), y_ref.view(np.uint32)), what
    abs_sum = oracle.reduce_fp(y_ref, "sum", 0.0, want_abs=True)[1] + abs(float(s0))
    return check_value(float(s_got), s_ref, abs_sum, synth.F32, "sum", str(what), n=y_ref.size)


def x_value(x: torch.Tensor):
    if x.dtype == torch.bfloat16:
        return float(x.float().item())
    return x.item()
