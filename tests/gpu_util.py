"""Helpers of the GPU parity tests: upload a synthetic problem and compare with the oracle."""
from __future__ import annotations

import numpy as np

import synth


def to_device(p: synth.Problem, row_major: bool = False, device="cuda"):
    """(Y, W) CUDA tensors of shape (m, n); column-major views unless row_major."""
    import torch
    if row_major:
        Y = torch.from_numpy(np.ascontiguousarray(p.Y)).to(device)
        W = torch.from_numpy(np.ascontiguousarray(p.W)).to(device)
    else:
        Y = torch.from_numpy(p.Yt).to(device).T
        W = torch.from_numpy(p.Wt.view(bool)).to(device).T
    return Y, W


def lower_N(N_tensor) -> np.ndarray:
    """The library's N (column-major, lower triangle written) as a full symmetric array."""
    A = N_tensor.detach().cpu().numpy().T  # column-major -> (i, j)
    L = np.tril(A)
    return L + np.tril(L, -1).T


def gamma(k: int, u: float) -> float:
    """Higham's gamma_k = k u / (1 - k u)."""
    return k * u / (1.0 - k * u)


def gram_bound_ok(G_gpu, Z, u, slack=2.0):
    """|G_gpu - Z^T Z| <= slack * gamma_{|R|+1}(u) |Z|^T |Z| elementwise (the dot-product bound)."""
    Z = np.asarray(Z, dtype=np.float64)
    ref = Z.T @ Z
    bound = slack * gamma(Z.shape[0] + 1, u) * (np.abs(Z).T @ np.abs(Z)) + 1e-300
    return np.all(np.abs(G_gpu - ref) <= bound), float(np.max(np.abs(G_gpu - ref) / bound))
