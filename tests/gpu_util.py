"""Helpers for the GPU parity tests (test-side only)."""
from __future__ import annotations

import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a: np.ndarray, dtype=torch.complex128) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().to(torch.complex128).cpu().numpy()


def assert_state_close(got: np.ndarray, want: np.ndarray, tol: float, what: str = "", l2tol: float | None = None):
    """Both bars: max |delta amplitude| <= tol and ||delta||_2 <= l2tol
    (default tol)."""
    d = got.astype(np.complex128) - want
    mx = float(np.max(np.abs(d))) if d.size else 0.0
    l2 = float(np.linalg.norm(d))
    l2tol = tol if l2tol is None else l2tol
    assert mx <= tol and l2 <= l2tol, "%s: max|d|=%.3e ||d||=%.3e tol=%.1e" % (what, mx, l2, tol)
    return mx, l2


def dense_from_dia(n: int, diags: dict) -> np.ndarray:
    N = 1 << n
    A = np.zeros((N, N), dtype=np.complex128)
    for d, v in diags.items():
        L = N - abs(d)
        t = np.arange(L)
        A[t + max(0, -d), t + max(0, d)] = v
    return A
