"""Error measures of Section 1.1 in FP64 (TEST INFRASTRUCTURE ONLY).

* cov-err(A, B)  = ||A^T A - B^T B||_2 / ||A||_F^2
* proj-err(A, B) = ||A - pi_{B_k}(A)||_F^2 / ||A - A_k||_F^2, with B_k the span
  of the top-k right singular vectors of B and A_k the best rank-k
  approximation of A (k = 10 by default, as in the experiments).
* proj-full(A, B) = ||A - pi_B(A)||_F^2 / ||A||_F^2, projecting on the whole
  row space of B (pi_X(A) = A X^+ X, Section 1.1).
"""
from __future__ import annotations

import numpy as np


def fro2(X: np.ndarray) -> float:
    X = np.asarray(X, dtype=np.float64)
    return float(np.sum(X * X))


def cov_err(A: np.ndarray, B: np.ndarray) -> float:
    """Spectral norm of A^T A - B^T B over ||A||_F^2 (dense eigvalsh)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    M = A.T @ A - B.T @ B
    w = np.linalg.eigvalsh(M)
    return float(max(abs(w[0]), abs(w[-1])) / fro2(A))


def _row_basis(B: np.ndarray, k: int | None = None, rtol: float = 1e-12):
    """Orthonormal rows spanning the top-k right singular directions of B."""
    B = np.asarray(B, dtype=np.float64)
    if B.size == 0:
        return np.zeros((0, B.shape[1]))
    _, s, vt = np.linalg.svd(B, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((0, B.shape[1]))
    rank = int(np.sum(s > rtol * s[0]))
    if k is not None:
        rank = min(rank, k)
    return vt[:rank]


def tail_mass(A: np.ndarray, k: int) -> float:
    """||A - A_k||_F^2 = sum of squared singular values of A beyond the k-th."""
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(np.sum(s[k:] ** 2))


def proj_err(A: np.ndarray, B: np.ndarray, k: int = 10) -> float:
    A = np.asarray(A, dtype=np.float64)
    V = _row_basis(B, k)
    num = fro2(A) - fro2(A @ V.T)
    den = tail_mass(A, k)
    return float(num / den) if den > 0 else float("nan")


def proj_full(A: np.ndarray, B: np.ndarray) -> float:
    A = np.asarray(A, dtype=np.float64)
    V = _row_basis(B)
    return float((fro2(A) - fro2(A @ V.T)) / fro2(A))


# Streams too long to hold as one matrix are scored from their column Gram
# A^T A, accumulated chunk by chunk.  The measure is the same definition
# (Section 1.1): the spectral norm of A^T A - B^T B over ||A||_F^2.

def gram(A: np.ndarray) -> np.ndarray:
    """A^T A in FP64."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def cov_err_gram(AtA: np.ndarray, fro2A: float, B: np.ndarray) -> float:
    """||A^T A - B^T B||_2 / ||A||_F^2 from A's column Gram (dense eigvalsh)."""
    B = np.asarray(B, dtype=np.float64)
    M = np.asarray(AtA, dtype=np.float64) - B.T @ B
    w = np.linalg.eigvalsh(M)
    return float(max(abs(w[0]), abs(w[-1])) / fro2A)
