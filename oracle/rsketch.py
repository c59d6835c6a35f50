"""Plain FP64 oracle of the paper's streaming hashing and sampling sketches
(TEST INFRASTRUCTURE ONLY: only the test-suite, the package smoke test and the
benchmark's CPU-baseline leg use it; it shares no code with the GPU path).

* Hashing (Section 2.2, "Sparse Random Projections"): B = S A with S an
  l x n matrix holding one nonzero per column, a random sign at a random row:
  row i of A is added, with sign sigma(i), to row h(i) of B.
* OSNAP (Section 2.2, same paragraph): s independent such matrices stacked,
  each with l/s rows.  Reading: every instance is scaled by 1/sqrt(s), so
  that B^T B estimates A^T A without bias (the text stacks the instances and
  states no scale).
* Priority sampling (Section 3.2, "Priority Sampling"): row i gets
  u_i ~ Unif(0,1), weight w_i = ||a_i||^2 and priority rho_i = w_i / u_i; the
  l rows of largest priority are kept, each with squared norm
  w^_i = max(w_i, tau).  Reading: tau is the (l+1)-th largest priority of the
  whole stream (0 when at most l rows arrived), the threshold under which
  every estimate w^_i is unbiased.
* VarOpt sampling (Section 3.2, "VarOpt Sampling"): the threshold tau solves
  sum_i min(1, w_i / tau) = l; item i is kept with probability
  p_i = min(1, w_i/tau) and given w^_i = max(w_i, tau), exactly l are kept,
  and sum over kept w^_i = ||A||_F^2.  The stream is taken in chunks: the
  reservoir (adjusted weights) and the chunk's rows are the candidates, the
  new threshold is that of the candidates, candidates at or above it stay,
  and the others are chosen by systematic sampling (one uniform offset per
  chunk, candidates in order: the reservoir's below-threshold rows, then the
  chunk's rows in stream order) with probabilities w^/tau, after which the
  chosen ones carry w^ = tau.  Reading: the paper fixes the inclusion
  probabilities, the sample size and the weight identity and leaves how the
  below-threshold rows are drawn; systematic sampling meets all three.

Random numbers come from a counter-based generator implemented here from its
published definition (SplitMix64, Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", 2014: add the golden-ratio increment, then
two xor-shift-multiply rounds and a final xor-shift):
  r(key, i, j) = mix(mix(key ^ i) ^ j), with mix(x) the SplitMix64 output
  for state x.
  * bucket of row i in hashing instance j: the high 32 bits of r(key, i, 2j),
    times the instance's rows, shifted right by 32;
  * sign of row i in instance j: - if the top bit of r(key, i, 2j+1) is set;
  * uniform of row i: (top 53 bits of r(key, i, 0) + 1/2) * 2^-53, in (0, 1);
  * systematic offset of VarOpt chunk c: the uniform of index 2^62 + c.
"""
from __future__ import annotations

import numpy as np

HASH, OSNAP, PRIORITY, VAROPT = "hash", "osnap", "priority", "varopt"
KINDS = (HASH, OSNAP, PRIORITY, VAROPT)

_M64 = (1 << 64) - 1
_INC = 0x9E3779B97F4A7C15
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB


def mix(x: int) -> int:
    """SplitMix64 output for state x (one step from state x - increment)."""
    z = (x + _INC) & _M64
    z = ((z ^ (z >> 30)) * _C1) & _M64
    z = ((z ^ (z >> 27)) * _C2) & _M64
    return z ^ (z >> 31)


def rbits(key: int, i: int, j: int) -> int:
    return mix(mix((key ^ i) & _M64) ^ j)


def bucket(key: int, i: int, inst: int, rows: int) -> int:
    return ((rbits(key, i, 2 * inst) >> 32) * rows) >> 32


def sign(key: int, i: int, inst: int) -> float:
    return -1.0 if rbits(key, i, 2 * inst + 1) >> 63 else 1.0


def uniform(key: int, i: int) -> float:
    return ((rbits(key, i, 0) >> 11) + 0.5) * 2.0 ** -53


def chunk_offset(key: int, c: int) -> float:
    return uniform(key, (1 << 62) + c)


class RSketchOracle:
    """Streaming oracle: append row blocks in order, then finalize()."""

    def __init__(self, kind: str, d: int, l: int, s: int = 4, key: int = 0):
        if kind not in KINDS:
            raise ValueError(kind)
        self.kind, self.d, self.l, self.s, self.key = kind, d, l, s, key
        self.n = 0
        self.fro2A = 0.0
        self.chunks = 0
        if kind in (HASH, OSNAP):
            self.inst = 1 if kind == HASH else s
            if l % self.inst:
                raise ValueError("OSNAP needs l divisible by s")
            self.B = np.zeros((l, d))
        else:
            self.rows = np.zeros((0, d))     # reservoir rows (as given, FP64)
            self.w = np.zeros(0)             # their squared norms
            self.what = np.zeros(0)          # adjusted weights (VarOpt)
            self.rho = np.zeros(0)           # priorities (Priority)
            self.idx = np.zeros(0, dtype=np.int64)
            self.tau = 0.0

    # -- Hashing / OSNAP: row i added to one row of each instance
    def _append_hash(self, X):
        rows = self.l // self.inst
        scale = 1.0 / np.sqrt(self.inst)
        for r in range(X.shape[0]):
            i = self.n + r
            for j in range(self.inst):
                b = j * rows + bucket(self.key, i, j, rows)
                self.B[b] += (sign(self.key, i, j) * X[r]) * scale

    # -- Priority: keep the l largest priorities; tau = largest one dropped
    def _append_priority(self, X):
        n0 = self.n
        w = np.einsum("ij,ij->i", X, X)
        u = np.array([uniform(self.key, n0 + r) for r in range(X.shape[0])])
        rho = w / u
        rows = np.vstack([self.rows, X])
        W = np.r_[self.w, w]
        R = np.r_[self.rho, rho]
        I = np.r_[self.idx, np.arange(n0, n0 + X.shape[0])]
        if R.size > self.l:
            order = np.argsort(-R, kind="stable")
            keep, drop = order[:self.l], order[self.l:]
            self.tau = max(self.tau, float(R[drop].max()))
            keep = np.sort(keep)
            rows, W, R, I = rows[keep], W[keep], R[keep], I[keep]
        self.rows, self.w, self.rho, self.idx = rows, W, R, I

    # -- VarOpt: threshold of the candidates, systematic choice below it
    @staticmethod
    def threshold(wh: np.ndarray, l: int) -> float:
        """tau with sum min(1, wh/tau) = l (the candidates number more than l):
        with the weights sorted in descending order, the first t are at or
        above tau and tau = (sum of the others) / (l - t)."""
        s = np.sort(wh)[::-1]
        tail = np.cumsum(s[::-1])[::-1]          # tail[t] = sum_{j >= t} s_j
        for t in range(l):
            tau = tail[t] / (l - t)
            if s[t] < tau:
                return float(tau)
        raise AssertionError("unreachable for more than l candidates")

    def _append_varopt(self, X):
        n0 = self.n
        w = np.einsum("ij,ij->i", X, X)
        rows = np.vstack([self.rows, X])
        W = np.r_[self.w, w]
        WH = np.r_[self.what, w]
        I = np.r_[self.idx, np.arange(n0, n0 + X.shape[0])]
        if WH.size > self.l:
            tau = self.threshold(WH, self.l)
            large = WH >= tau
            t = int(large.sum())
            small = np.flatnonzero(~large)           # reservoir's first, then the chunk's
            p = WH[small] / tau
            C = np.cumsum(p)
            u = chunk_offset(self.key, self.chunks)
            k = self.l - t
            # Positions (q + u) C_total / k, q = 0..k-1, each in the interval
            # (C_{j-1}, C_j] of one small candidate.
            pos = (np.arange(k) + u) * (C[-1] / k)
            pick = small[np.searchsorted(C, pos, side="left")]
            assert np.unique(pick).size == k
            keep = np.sort(np.r_[np.flatnonzero(large), pick])
            WH = WH.copy()
            WH[pick] = tau
            rows, W, WH, I = rows[keep], W[keep], WH[keep], I[keep]
            self.tau = tau
        self.rows, self.w, self.what, self.idx = rows, W, WH, I

    def append(self, X: np.ndarray):
        X = np.asarray(X, dtype=np.float64)
        if X.shape[0] == 0:
            return self
        self.fro2A += float(np.sum(X * X))
        if self.kind in (HASH, OSNAP):
            self._append_hash(X)
        elif self.kind == PRIORITY:
            self._append_priority(X)
        else:
            self._append_varopt(X)
        self.n += X.shape[0]
        self.chunks += 1
        return self

    def finalize(self) -> np.ndarray:
        """The l x d sketch (zero rows where fewer than l were kept)."""
        if self.kind in (HASH, OSNAP):
            return self.B.copy()
        B = np.zeros((self.l, self.d))
        if self.kind == PRIORITY:
            wh = np.maximum(self.w, self.tau)
        else:
            wh = self.what
        k = self.rows.shape[0]
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.where(self.w > 0, np.sqrt(wh / np.where(self.w > 0, self.w, 1.0)), 0.0)
        B[:k] = self.rows * f[:, None]
        return B

    def adjusted_weights(self) -> np.ndarray:
        if self.kind == PRIORITY:
            return np.maximum(self.w, self.tau)
        if self.kind == VAROPT:
            return self.what.copy()
        raise ValueError("sampling sketches only")


def rsketch(A: np.ndarray, kind: str, l: int, s: int = 4, key: int = 0, chunks=None):
    """Sketch A in one pass (rows appended in the given chunk sizes)."""
    sk = RSketchOracle(kind, A.shape[1], l, s, key)
    if chunks is None:
        sk.append(A)
    else:
        lo = 0
        for c in chunks:
            sk.append(A[lo:lo + c])
            lo += c
        sk.append(A[lo:])
    return sk.finalize(), sk
