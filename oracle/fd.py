"""Plain FP64 oracle of the Frequent Directions family (TEST INFRASTRUCTURE ONLY).

Follows the generic iterative sketch of Section 2.3 (Algorithm 1): rows are
written into free rows of a buffer; when the buffer is full its SVD
B = U S V^T is taken, the singular values are changed by a ReduceRank rule and
the buffer becomes S' V^T.  The rules:

* FD (Section 2.3, "Frequent Directions", with Liberty's fast variant):
  delta = sigma_l^2, sigma'_j^2 = max(sigma_j^2 - delta, 0) for every j.
* iSVD (Section 2.3, "Iterative SVD"): sigma'_j = sigma_j for j < l and
  sigma'_j = 0 from j = l on.  The value sigma_l^2 is recorded as delta.
* alpha-FD (Section 3.1, Algorithm 2, ReduceRank-PFD): delta = sigma_l^2, the
  leading l(1-alpha) values are untouched, the trailing alpha*l are shrunk.
* fast alpha-FD (Section 3.1, "Fast Parameterized FD"): delta = sigma_t^2 with
  t = l - alpha*l/2, only the trailing alpha*l values are shrunk, clamped at 0.

Readings taken where the text is silent or inexact (each is listed with its
reason in the design notes):

1. The buffer has m rows (m = 2l by default, m = l reproduces Algorithm 1
   literally); the rules are evaluated with the sketch size l, singular values
   are padded with zeros up to m, and shrunk values are clamped at zero.
2. s = ceil(alpha*l) trailing values are shrunk, r = l - s are untouched; the
   fast variant uses t = r + ceil(s/2).
3. The schedule is data independent: after a ReduceRank the first t-1 rows
   count as occupied (even when some are zero), the next rows go after them,
   and a ReduceRank runs whenever all m rows are occupied.
4. At the end, if more than l rows are occupied one more ReduceRank runs; the
   sketch is the first l rows of the buffer.

The SVD route here (LAPACK gesdd on the m x d buffer) is deliberately a
different algorithm from the GPU path's Gram matrix + Jacobi eigensolver.
"""
from __future__ import annotations

import math

import numpy as np

FD, ISVD, ALPHA, FAST_ALPHA = "fd", "isvd", "alpha", "fast_alpha"
VARIANTS = (FD, ISVD, ALPHA, FAST_ALPHA)


def _split(l: int, alpha: float):
    """s = ceil(alpha*l) shrunk values, r = l - s untouched (reading 2)."""
    if not (0.0 < alpha <= 1.0):
        raise ValueError("alpha must lie in (0, 1]")
    s = int(math.ceil(alpha * l * (1.0 - 1e-12)))
    s = min(max(s, 1), l)
    return l - s, s


def rule_indices(l: int, variant: str, alpha: float = 0.2):
    """Return (t, r): delta = sigma_t^2 (1-based t), r leading values untouched.

    After a ReduceRank rows t, t+1, ... of S'V^T are zero, so t-1 rows survive.
    """
    if variant == FD:
        return l, 0
    if variant == ISVD:
        return l, l - 1
    r, s = _split(l, alpha)
    if variant == ALPHA:
        return l, r
    if variant == FAST_ALPHA:
        return r + (s + 1) // 2, r
    raise ValueError(f"unknown variant {variant!r}")


def alpha_eff(l: int, variant: str, alpha: float = 0.2) -> float:
    """Constant of Property 3 (mass removed >= alpha_eff * l * Delta)."""
    if variant == FD:
        return 1.0
    if variant == ISVD:
        return 1.0 / l
    r, s = _split(l, alpha)
    if variant == ALPHA:
        return s / l
    t, _ = rule_indices(l, variant, alpha)
    return (t - r) / l


def reduce_rank(sigma: np.ndarray, l: int, variant: str, alpha: float = 0.2):
    """Apply one ReduceRank rule to descending singular values (length >= l).

    Returns (sigma_new, delta).
    """
    lam = np.asarray(sigma, dtype=np.float64) ** 2
    t, r = rule_indices(l, variant, alpha)
    delta = lam[t - 1]
    if variant == ISVD:
        lam_new = lam.copy()
        lam_new[l - 1:] = 0.0
    else:
        lam_new = lam.copy()
        lam_new[r:] = np.maximum(lam[r:] - delta, 0.0)
    return np.sqrt(lam_new), float(delta)


class SketchOracle:
    """Streaming sketch state: buffer, occupancy and the FP64 accumulators."""

    def __init__(self, d: int, l: int, variant: str = FD, alpha: float = 0.2,
                 m: int | None = None):
        if l < 1 or d < 1:
            raise ValueError("need l >= 1 and d >= 1")
        self.d, self.l, self.variant, self.alpha = d, l, variant, alpha
        self.m = 2 * l if m is None else int(m)
        if self.m < l:
            raise ValueError("buffer must have at least l rows")
        self.t, self.r = rule_indices(l, variant, alpha)
        self.C = np.zeros((self.m, d))
        self.occ = 0
        self.fro2A = 0.0      # ||A||_F^2 of everything appended
        self.Delta = 0.0      # sum of delta_i (Section 3.1)
        self.Stot = 0.0       # total squared mass removed by the rules
        self.n_rows = 0
        self.n_rr = 0

    def _reduce(self):
        _, sig, vt = np.linalg.svd(self.C[:self.occ], full_matrices=False)
        sig_full = np.zeros(max(self.m, self.l))
        sig_full[:sig.size] = sig
        sig_new, delta = reduce_rank(sig_full, self.l, self.variant, self.alpha)
        keep = self.t - 1
        C = np.zeros_like(self.C)
        kk = min(keep, vt.shape[0])
        C[:kk] = sig_new[:kk, None] * vt[:kk]
        self.Stot += float(np.sum(sig_full ** 2 - sig_new ** 2))
        self.Delta += delta
        self.n_rr += 1
        self.C = C
        self.occ = keep

    def append(self, rows: np.ndarray):
        rows = np.atleast_2d(np.asarray(rows, dtype=np.float64))
        i = 0
        while i < rows.shape[0]:
            f = min(self.m - self.occ, rows.shape[0] - i)
            block = rows[i:i + f]
            self.C[self.occ:self.occ + f] = block
            self.fro2A += float(np.sum(block * block))
            self.occ += f
            self.n_rows += f
            i += f
            if self.occ == self.m:
                self._reduce()

    def finalize(self) -> np.ndarray:
        if self.occ > self.l:
            self._reduce()
        return self.C[:self.l].copy()

    def stats(self) -> dict:
        return dict(fro2A=self.fro2A, Delta=self.Delta, Stot=self.Stot,
                    n_rows=self.n_rows, n_rr=self.n_rr, occ=self.occ)


def fd_sketch(A: np.ndarray, l: int, variant: str = FD, alpha: float = 0.2,
              m: int | None = None, return_state: bool = False):
    """Sketch every row of A; return the l x d sketch (and the oracle state)."""
    A = np.asarray(A)
    sk = SketchOracle(A.shape[1], l, variant, alpha, m)
    sk.append(A)
    B = sk.finalize()
    return (B, sk) if return_state else B


def fd_covariance_form(A: np.ndarray, l: int, variant: str = FD, alpha: float = 0.2,
                       m: int | None = None) -> np.ndarray:
    """Independent re-derivation of B^T B through d x d eigendecompositions.

    Keeps only M = B^T B.  At each scheduled ReduceRank the buffer's covariance
    is K = M + X^T X (X = rows appended since the last one); its eigenvalues are
    the squared singular values of the buffer, so applying the rule to them
    and rebuilding V diag(.) V^T gives the next M.  Intended for small d.
    """
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    mm = 2 * l if m is None else m
    t, r = rule_indices(l, variant, alpha)
    M = np.zeros((d, d))
    occ, i = 0, 0
    pending = np.zeros((0, d))

    def reduce(M, pending):
        K = M + pending.T @ pending
        w, V = np.linalg.eigh(K)
        w, V = w[::-1], V[:, ::-1]
        top = np.zeros(max(mm, l))
        kk = min(mm, d)
        top[:kk] = np.maximum(w[:kk], 0.0)
        lam = top.copy()
        delta = top[t - 1]
        if variant == ISVD:
            lam[l - 1:] = 0.0
        else:
            lam[r:] = np.maximum(top[r:] - delta, 0.0)
        return (V[:, :kk] * lam[:kk]) @ V[:, :kk].T

    while i < n:
        f = min(mm - occ, n - i)
        pending = np.vstack([pending, A[i:i + f]])
        occ += f
        i += f
        if occ == mm:
            M = reduce(M, pending)
            pending = np.zeros((0, d))
            occ = t - 1
    if occ > l:
        M = reduce(M, pending)
    else:
        M = M + pending.T @ pending
    return M


def counter_simulation(j: np.ndarray, c: np.ndarray, d: int, l: int,
                       variant: str = FD, alpha: float = 0.2, m: int | None = None):
    """Frequent-items view of the sketch for rows c_i * e_{j_i} (Section 1.2).

    For such rows the buffer's right singular vectors are coordinate vectors
    and its squared singular values are per-coordinate squared-weight totals,
    so the sketch reduces to a weighted Misra-Gries summary: counters of
    squared weight, and at each scheduled reduction the l-th largest total is
    subtracted from every counter (clamped at zero) -- or, for the variants,
    from the trailing counters only / the trailing ones are dropped.
    Returns the diagonal of B^T B.
    """
    mm = 2 * l if m is None else m
    counters = np.zeros(d)
    pending = np.zeros(d)
    occ = 0
    if variant == FD:
        keep_top, t = 0, l
    elif variant == ISVD:
        keep_top, t = l - 1, l
    else:
        s = min(max(int(math.ceil(alpha * l * (1.0 - 1e-12))), 1), l)
        keep_top = l - s
        t = l if variant == ALPHA else keep_top + (s + 1) // 2

    def reduce(counters, pending):
        totals = counters + pending
        order = np.argsort(-totals, kind="stable")
        ranked = totals[order]
        ranked = np.concatenate([ranked, np.zeros(max(0, mm - ranked.size))])
        cut = ranked[t - 1]
        new = totals.copy()
        for rank, idx in enumerate(order):
            if variant == ISVD:
                if rank >= l - 1:
                    new[idx] = 0.0
            elif rank >= keep_top:
                new[idx] = max(totals[idx] - cut, 0.0)
        return new

    for jj, cc in zip(j, c):
        pending[jj] += cc * cc
        occ += 1
        if occ == mm:
            counters = reduce(counters, pending)
            pending[:] = 0.0
            occ = t - 1
    if occ > l:
        counters = reduce(counters, pending)
    else:
        counters = counters + pending
    return counters
