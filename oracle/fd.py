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
* SpaceSaving Directions (Section 3.1, Algorithm 3): delta = sigma_{l-1}^2;
  sigma_{l-1} becomes 0 and sigma_l becomes sqrt(sigma_l^2 + delta), the
  others are untouched.  Algorithm 3 returns exactly l values, so SSD runs on
  the l-row buffer of Algorithm 1 (m = l).
* Compensative FD (Section 3.1, "Compensative Frequent Directions"): FD
  during the stream; at the end B = S' V^T of the latest reduction is
  returned with each of the l output squared singular values raised by
  Delta = sum of all delta_i (so the l-th direction, zeroed by that
  reduction, carries sqrt(Delta)).  When rows arrived after the latest
  reduction, the buffer's own SVD (after one more FD reduction if more than
  l rows are occupied) plays that role.

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
5. A direction with a zero singular value (at or below 1e-12 of the largest
   squared one before the reduction) is not in the buffer's row space: SSD
   then has nothing to move and leaves the values unchanged (delta = 0), and
   CFD leaves that output row zero.
6. Merge: another sketch's occupied buffer rows are inserted
   like stream rows without counting into ||A||_F^2, and its accumulators
   (||A||_F^2, Delta, S_tot, rows, reductions) are added.

The SVD route here (LAPACK gesdd on the m x d buffer) is deliberately a
different algorithm from the GPU path's Gram matrix + Jacobi eigensolver.
"""
from __future__ import annotations

import math

import numpy as np

FD, ISVD, ALPHA, FAST_ALPHA = "fd", "isvd", "alpha", "fast_alpha"
SSD, CFD = "ssd", "cfd"
VARIANTS = (FD, ISVD, ALPHA, FAST_ALPHA)
ALL_VARIANTS = VARIANTS + (SSD, CFD)
NULL_REL = 1e-12        # squared singular values at or below this times the largest are zero (reading 5)


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
    if variant in (FD, CFD, SSD):
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
    if variant in (FD, CFD):
        return 1.0
    if variant == ISVD:
        return 1.0 / l
    if variant == SSD:
        raise ValueError("SSD does not satisfy Property 3 as it stands (its mass is conserved)")
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
    if variant == SSD:
        lam_new = lam.copy()
        if lam[l - 1] <= NULL_REL * lam[0]:
            return np.sqrt(lam_new), 0.0           # a free direction: nothing to move
        delta = lam[l - 2]
        lam_new[l - 2] = 0.0
        lam_new[l - 1] = lam[l - 1] + delta
        return np.sqrt(lam_new), float(delta)
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
        if variant == SSD and (self.m != l or l < 2):
            raise ValueError("SSD runs on an l-row buffer with l >= 2")
        self.t, self.r = rule_indices(l, variant, alpha)
        self.C = np.zeros((self.m, d))
        self.occ = 0
        self.fro2A = 0.0      # ||A||_F^2 of everything appended
        self.Delta = 0.0      # sum of delta_i (Section 3.1)
        self.Stot = 0.0       # total squared mass removed by the rules
        self.n_rows = 0
        self.n_rr = 0
        self._last = None         # (lambda, lambda', V^T) of the latest ReduceRank
        self._since = 0           # rows appended since it

    def _reduce(self):
        _, sig, vt = np.linalg.svd(self.C[:self.occ], full_matrices=False)
        sig_full = np.zeros(max(self.m, self.l))
        sig_full[:sig.size] = sig
        sig_new, delta = reduce_rank(sig_full, self.l, self.variant, self.alpha)
        keep = self.t - 1
        C = np.zeros_like(self.C)
        rows = list(range(keep))
        if self.variant == SSD and delta > 0.0:
            rows[self.l - 2] = self.l - 1           # the merged direction takes the freed slot
        for q, j in enumerate(rows):
            if j < vt.shape[0]:
                C[q] = sig_new[j] * vt[j]
        self.Stot += float(np.sum(sig_full ** 2 - sig_new ** 2))
        self.Delta += delta
        self.n_rr += 1
        self.C = C
        self.occ = keep
        self._last = (sig_full ** 2, sig_new ** 2, vt)   # for Compensative FD's last step

    def append(self, rows: np.ndarray):
        self._insert(rows, count=True)

    def _insert(self, rows, count):
        """Algorithm 1's insertion; `count` adds the rows to ||A||_F^2 and the
        row count (they are stream rows rather than another sketch's)."""
        rows = np.atleast_2d(np.asarray(rows, dtype=np.float64))
        i = 0
        while i < rows.shape[0]:
            f = min(self.m - self.occ, rows.shape[0] - i)
            block = rows[i:i + f]
            self.C[self.occ:self.occ + f] = block
            if count:
                self.fro2A += float(np.sum(block * block))
                self.n_rows += f
            self.occ += f
            self._since += f
            i += f
            if self.occ == self.m:
                self._reduce()
                self._since = 0

    def merge(self, other: "SketchOracle"):
        """Absorb another sketch of the same configuration (reading 6): its
        occupied buffer rows are inserted like stream rows, without counting
        them into ||A||_F^2, and its accumulators are added.  By the argument
        of the three-property framework (Section 3.1), the result sketches
        the union of the two streams with Delta = Delta_1 + Delta_2 + the
        merge's own."""
        if (other.d, other.l, other.variant, other.m) != (self.d, self.l, self.variant, self.m):
            raise ValueError("merge needs sketches of the same configuration")
        if self.variant in (ALPHA, FAST_ALPHA) and other.alpha != self.alpha:
            raise ValueError("merge needs the same alpha")
        rows = other.C[:other.occ].copy()
        fro2A, Delta, Stot = other.fro2A, other.Delta, other.Stot
        n_rows, n_rr = other.n_rows, other.n_rr
        self._insert(rows, count=False)
        self.fro2A += fro2A
        self.Delta += Delta
        self.Stot += Stot
        self.n_rows += n_rows
        self.n_rr += n_rr

    def finalize(self) -> np.ndarray:
        if self.variant == CFD:
            return self._finalize_cfd()
        if self.occ > self.l:
            self._reduce()
        return self.C[:self.l].copy()

    def _finalize_cfd(self) -> np.ndarray:
        """Compensative FD's last step: B = S' V^T of the latest reduction with
        sigma_hat_j = sqrt(sigma'_j^2 + Delta) for the l output rows (Delta the
        total subtracted).  When rows arrived after the latest reduction (or
        none ran), the buffer's own SVD is that S' V^T, after one more FD
        reduction if more than l rows are occupied."""
        l = self.l
        if self._last is not None and self._since == 0:
            lam, lam_new, vt = self._last
            kept = float(np.sum(lam_new))               # mass the buffer holds now
        else:
            _, sig, vt = np.linalg.svd(self.C[:self.occ], full_matrices=False)
            lam = np.zeros(max(self.m, l))
            lam[:sig.size] = sig ** 2
            lam_new = lam.copy()
            kept = float(np.sum(lam))
            if self.occ > l:
                delta = lam[l - 1]
                lam_new = np.maximum(lam - delta, 0.0)
                self.Delta += delta
                self.n_rr += 1
        out = np.zeros((l, self.d))
        written = 0.0
        for j in range(min(l, vt.shape[0])):
            if lam[j] > NULL_REL * lam[0]:
                out[j] = np.sqrt(lam_new[j] + self.Delta) * vt[j]
                written += lam_new[j] + self.Delta
        self.Stot += kept - written
        self.C = np.zeros_like(self.C)
        self.C[:l] = out
        self.occ = l
        return out.copy()

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
    if variant == SSD:
        return _counter_ssd(j, c, d, l)
    if variant == CFD:
        return _counter_cfd(j, c, d, l, mm)
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


def _counter_ssd(j, c, d, l):
    """SpaceSaving on squared-weight counters (l-row buffer): after l rows, the
    two smallest of the l largest totals merge -- the second smallest is
    emptied into the smallest -- unless the smallest is empty."""
    counters = np.zeros(d)
    occ = 0
    for jj, cc in zip(j, c):
        counters[jj] += cc * cc
        occ += 1
        if occ == l:
            order = np.argsort(-counters, kind="stable")
            top = counters[order[0]]
            a, b = order[l - 2], order[l - 1]        # ranks l-1 and l (1-based)
            if counters[b] > NULL_REL * top:
                counters[b] += counters[a]
                counters[a] = 0.0
            else:
                counters[b] = 0.0
            occ = l - 1
    return counters


def _counter_cfd(j, c, d, l, mm):
    """Compensative FD on counters: the FD simulation, then Delta added to each
    of the (at most l) largest non-empty totals at the end."""
    counters = np.zeros(d)
    pending = np.zeros(d)
    occ, Delta = 0, 0.0

    def ranked_cut(totals):
        r = np.sort(totals)[::-1]
        r = np.concatenate([r, np.zeros(max(0, mm - r.size))])
        return r[l - 1]

    last = None
    since = 0
    for jj, cc in zip(j, c):
        pending[jj] += cc * cc
        occ += 1
        since += 1
        if occ == mm:
            totals = counters + pending
            cut = ranked_cut(totals)
            counters = np.maximum(totals - cut, 0.0)
            Delta += cut
            last = (totals, counters.copy())
            pending[:] = 0.0
            occ = l - 1
            since = 0
    if last is not None and since == 0:
        totals, shrunk = last
    else:
        totals = counters + pending
        if occ > l:
            cut = ranked_cut(totals)
            shrunk = np.maximum(totals - cut, 0.0)
            Delta += cut
        else:
            shrunk = totals
    order = np.argsort(-totals, kind="stable")
    out = np.zeros(d)
    top = totals[order[0]] if d else 0.0
    for idx in order[:l]:
        if totals[idx] > NULL_REL * top:
            out[idx] = shrunk[idx] + Delta
    return out
