"""Helpers shared by the GPU parity tests: oracle references and error norms."""
import numpy as np
import torch

import oracle


def abs_csr(A):
    return oracle.CSR(A.n, A.rowptr, A.col, np.abs(A.val))


def stage_bound_apply(A, T, u):
    """Elementwise forward-error bound for F = A T with unit roundoff u:
    7 products and 6 additions, bound (7 u + u) |A| |T| per entry."""
    return (8.0 * u) * oracle.apply_many(abs_csr(A), np.abs(T))


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_np(t):
    return t.detach().to(torch.float64).cpu().numpy()


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (through float32, nearest-even)."""
    t = torch.as_tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16)
    return t.to(torch.float64).numpy()


def f32_round(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)
