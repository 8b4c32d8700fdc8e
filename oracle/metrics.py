"""Parity metrics between two RSM results (test infrastructure only).

* Largest principal angle between column spaces, in the sine form
  theta_max = arcsin(min(1, ||B - A (A^T B)||_2)) for orthonormal A, B.  The cosine
  form arccos(sigma_min(A^T B)) cannot resolve angles below about 1e-8 in FP64.
* Relative RMS of the two low-rank products on the known entries,
  ||W o (U1 V1^T - U2 V2^T)||_F / ||W o U2 V2^T||_F, which does not depend on the
  basis chosen for V-hat because U-hat follows any rotation of it.
"""
from __future__ import annotations

import numpy as np


def orthonormal(A: np.ndarray) -> np.ndarray:
    q, _ = np.linalg.qr(np.asarray(A, dtype=np.float64))
    return q


def principal_angle_max(A: np.ndarray, B: np.ndarray) -> float:
    """Largest principal angle (radians) between span(A) and span(B) (sine form)."""
    A = orthonormal(A)
    B = orthonormal(B)
    if A.shape != B.shape:
        raise ValueError("subspaces of different dimension")
    resid = B - A @ (A.T @ B)
    s = np.linalg.norm(resid, 2)
    return float(np.arcsin(min(1.0, s)))


def principal_angle_max_cos(A: np.ndarray, B: np.ndarray) -> float:
    """The same angle from the cosine form (for cross-checks at angles well above 1e-8)."""
    A = orthonormal(A)
    B = orthonormal(B)
    sv = np.linalg.svd(A.T @ B, compute_uv=False)
    return float(np.arccos(min(1.0, sv.min())))


def rel_rms_known(W, U1, V1, U2, V2, block: int = 8192) -> float:
    """||W o (U1 V1^T - U2 V2^T)||_F / ||W o U2 V2^T||_F, one row block at a time."""
    W = np.asarray(W, dtype=bool)
    num = 0.0
    den = 0.0
    for i0 in range(0, W.shape[0], block):
        i1 = min(W.shape[0], i0 + block)
        P1 = U1[i0:i1] @ V1.T
        P2 = U2[i0:i1] @ V2.T
        Wb = W[i0:i1]
        num += float(np.sum(np.where(Wb, P1 - P2, 0.0) ** 2))
        den += float(np.sum(np.where(Wb, P2, 0.0) ** 2))
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))
