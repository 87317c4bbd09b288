"""Helpers shared by the GPU parity tests: device inputs, host copies for
the oracle, and the tolerance rules.

FP32/BF16 sums: |got - ref| <= 1e-6 |ref| (ref = FP64 oracle), or, when the
exact sum is 0, |got| <= 1e-6 * sum|x|.  FP64 sums: 1e-12 relative.
Integers, max/min and iteration maps: bit-exact.
"""
from __future__ import annotations

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


def check_value(got, ref, abs_sum, dtype: int, op: str, what: str = ""):
    if dtype in (synth.I32, synth.I64) or op != "sum":
        if op != "sum" and dtype not in (synth.I32, synth.I64):
            assert float(got) == float(ref), (what, got, ref)
        else:
            assert int(got) == int(ref), (what, got, ref)
        return
    tol = TOL_F64 if dtype == synth.F64 else TOL_F32
    if ref == 0.0:
        assert abs(float(got)) <= tol * abs_sum, (what, got, ref)
    else:
        assert abs(float(got) - ref) <= tol * abs(ref), (what, got, ref, abs(float(got) - ref) / abs(ref))


def x_value(x: torch.Tensor):
    if x.dtype == torch.bfloat16:
        return float(x.float().item())
    return x.item()
