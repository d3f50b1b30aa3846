"""torch-tensor convenience over the C ABI: allocation and stream plumbing only."""
from __future__ import annotations

import torch

from . import paco

_plans = {}


def get_plan(N1: int, N2: int, p: int, b: int, dt: int = paco.PACO_C64, mixed: bool = False) -> paco.Plan:
    """A cached plan per (device, N1, N2, p, b, dtype, mixed radix)."""
    key = (torch.cuda.current_device(), N1, N2, p, b, dt, mixed)
    plan = _plans.get(key)
    if plan is None:
        plan = _plans[key] = paco.Plan(N1, N2, p, b, dt, mixed=mixed)
    return plan


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check_tensor(x: torch.Tensor, n: int, name: str):
    if not x.is_cuda or x.dtype != torch.complex64 or not x.is_contiguous() or x.numel() != n:
        raise ValueError(f"{name} must be a contiguous complex64 CUDA tensor of {n} items")


def _run(method: str, x, N1, N2, p, b, dt, mixed, out, workspace):
    N = N1 * N2
    _check_tensor(x, N, "x")
    plan = get_plan(N1, N2, p, b, dt, mixed)
    if out is None:
        out = torch.empty(N, dtype=torch.complex64, device=x.device)
    _check_tensor(out, N, "out")
    if workspace is None:
        workspace = torch.empty(N, dtype=torch.complex64, device=x.device)
    getattr(plan, method)(x.data_ptr(), out.data_ptr(), workspace.data_ptr(), _stream())
    return out


def fft(x: torch.Tensor, N1: int, N2: int, p: int, b: int, out: torch.Tensor | None = None,
        workspace: torch.Tensor | None = None, dt: int = paco.PACO_C64, mixed: bool = False,
        two_pass: bool = False) -> torch.Tensor:
    """y = Omega_N x for x of N = N1*N2 items (viewed N1 x N2); returns y
    (the N2 x N1 factor-swapped view, flattened, is y in natural order).
    dt: butterfly arithmetic (PACO_C64 or a split MFMA form); mixed: sizes
    that are not powers of b; two_pass: the two-HBM-pass form."""
    return _run("execute_two_pass" if two_pass else "execute", x, N1, N2, p, b, dt, mixed, out, workspace)


def ifft(y: torch.Tensor, N1: int, N2: int, p: int, b: int, out: torch.Tensor | None = None,
         workspace: torch.Tensor | None = None, dt: int = paco.PACO_C64, mixed: bool = False) -> torch.Tensor:
    """x = Omega_N^{-1} y (scaled by 1/N) for y in natural order, with the
    forward plan's (N1, N2, p, b): the inverse of fft()."""
    return _run("execute_inverse", y, N1, N2, p, b, dt, mixed, out, workspace)


def stage(x: torch.Tensor, N1: int, N2: int, p: int, b: int, stage: int, flags: int = 0,
          out: torch.Tensor | None = None) -> torch.Tensor:
    """One phase alone (paco_execute_stage)."""
    N = N1 * N2
    _check_tensor(x, N, "x")
    plan = get_plan(N1, N2, p, b)
    if out is None:
        out = torch.empty(N, dtype=torch.complex64, device=x.device)
    plan.execute_stage(stage, x.data_ptr(), out.data_ptr(), _stream(), flags)
    return out


def fft_batched(x: torch.Tensor, plan: paco.BatchPlan, out: torch.Tensor | None = None,
                workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Every transform of a batch plan in one launch: x holds the inputs back
    to back (transform i at plan.offsets[i]); returns the outputs in the same
    places, each y_i in natural order."""
    _check_tensor(x, plan.total, "x")
    if out is None:
        out = torch.empty(plan.total, dtype=torch.complex64, device=x.device)
    _check_tensor(out, plan.total, "out")
    if workspace is None:
        workspace = torch.empty(plan.total, dtype=torch.complex64, device=x.device)
    plan.execute(x.data_ptr(), out.data_ptr(), workspace.data_ptr(), _stream())
    return out
