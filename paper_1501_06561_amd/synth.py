"""Seeded synthetic row streams for the Frequent Directions workloads.

This module only draws inputs.  It holds none of the sketching arithmetic, so
both the GPU path and the CPU oracle can consume what it produces.

Recipes
-------
* ``random_noisy`` -- the "Random Noisy" construction of the paper's dataset
  section (Section 4): A = S D U + N / zeta, S iid N(0,1) (n x k), D diagonal
  with linearly decreasing entries D_ii = 1 - (i-1)/k, U a k x d matrix with
  orthonormal rows (transpose of the reduced QR factor of a d x k Gaussian),
  N iid N(0,1).  The text prints the decay as (i-1)/d; with /k the generator
  reproduces the numeric rank the paper's dataset table lists, so /k is used.
  Draw order is fixed: S, then the Gaussian behind U, then N.
* ``power_law`` -- A = S diag(sigma) V^T + E with sigma_i = i^-p, S iid N(0,1)
  (n x r), V d x r with orthonormal columns, E iid N(0, noise_var).
* ``rotating_adversarial`` -- a stream whose dominant direction turns by a
  fixed angle every block of rows: row = g u_b + N / zeta.
* ``two_subspace_adversarial`` -- the paper's "Adversarial" construction
  (Section 4): Gaussian vectors projected on a first coordinate subspace, then
  on a second, disjoint one; every row normalised; all first-subspace rows
  come first.
* ``basis_rows`` -- rows that are scaled coordinate vectors (frequent-items
  special case used to test the sketch against a counter simulation).
* ``batch_shapes`` -- per-sketch (d, l, n) draws for the many-sketch workload;
  ``batch_sketch_rows`` -- the rows of one of its sketches.
* ``random_noisy_device`` -- the Random Noisy recipe drawn on a torch device
  (S and N from a seeded ``torch.Generator`` there, U from NumPy as above),
  for workloads too large to draw on the host quickly.

All NumPy draws use ``numpy.random.Generator(PCG64)``; chunked streams derive
one child seed per chunk so any chunk regenerates on its own.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for", "random_noisy", "random_noisy_chunk", "random_noisy_basis",
    "power_law", "power_law_basis", "power_law_chunk",
    "rotating_adversarial", "two_subspace_adversarial", "basis_rows",
    "batch_shapes", "batch_sketch_rows", "chunk_sizes", "parallel_map", "random_noisy_device",
    "to_bf16", "bf16_bits", "WORKLOADS",
]


def rng_for(*key: int) -> np.random.Generator:
    """Generator seeded by SeedSequence(key) (a single int key -> that seed)."""
    if len(key) == 1:
        return np.random.default_rng(key[0])
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _orthonormal_rows(rng: np.random.Generator, k: int, d: int) -> np.ndarray:
    g = rng.standard_normal((d, k))
    q, _ = np.linalg.qr(g)          # d x k, orthonormal columns
    return np.ascontiguousarray(q.T)  # k x d, orthonormal rows


def random_noisy(n: int, d: int, k: int, zeta: float = 10.0, seed=0,
                 dtype=np.float64) -> np.ndarray:
    """Random Noisy matrix, n x d, signal rank k (see module docstring)."""
    rng = rng_for(*seed) if isinstance(seed, (tuple, list)) else rng_for(seed)
    S = rng.standard_normal((n, k))
    U = _orthonormal_rows(rng, k, d)
    D = 1.0 - np.arange(k, dtype=np.float64) / k
    N = rng.standard_normal((n, d))
    A = (S * D) @ U + N / zeta
    return A.astype(dtype, copy=False)


def random_noisy_basis(d: int, k: int, seed_key) -> np.ndarray:
    """The k x d orthonormal-row factor U shared by every chunk of a stream."""
    return _orthonormal_rows(rng_for(*seed_key), k, d)


def random_noisy_chunk(U: np.ndarray, rows: int, zeta: float, seed_key,
                       dtype=np.float32) -> np.ndarray:
    """One chunk of a long Random Noisy stream (own child seed per chunk)."""
    k, d = U.shape
    rng = rng_for(*seed_key)
    S = rng.standard_normal((rows, k))
    D = 1.0 - np.arange(k, dtype=np.float64) / k
    N = rng.standard_normal((rows, d))
    return ((S * D) @ U + N / zeta).astype(dtype, copy=False)


def power_law_basis(d: int, r: int, seed_key) -> np.ndarray:
    """d x r orthonormal columns for the power-law workload."""
    g = rng_for(*seed_key).standard_normal((d, r))
    q, _ = np.linalg.qr(g)
    return np.ascontiguousarray(q)


def power_law_chunk(V: np.ndarray, rows: int, exponent: float, noise_var: float,
                    seed_key, dtype=np.float32) -> np.ndarray:
    d, r = V.shape
    rng = rng_for(*seed_key)
    S = rng.standard_normal((rows, r))
    sig = np.arange(1, r + 1, dtype=np.float64) ** (-exponent)
    E = rng.standard_normal((rows, d)) * np.sqrt(noise_var)
    return ((S * sig) @ V.T + E).astype(dtype, copy=False)


def power_law(n: int, d: int, r: int = 300, exponent: float = 0.8,
              noise_var: float = 1e-2, seed=(3, 0), chunk: int = 50_000,
              dtype=np.float32) -> np.ndarray:
    """Power-law spectrum matrix, generated chunk by chunk (child seeds)."""
    V = power_law_basis(d, r, tuple(seed))
    out = np.empty((n, d), dtype=dtype)
    for c, r0 in enumerate(range(0, n, chunk)):
        rows = min(chunk, n - r0)
        out[r0:r0 + rows] = power_law_chunk(V, rows, exponent, noise_var,
                                            tuple(seed) + (c + 1,), dtype)
    return out


def rotating_adversarial(n_blocks: int = 200, block_rows: int = 500, d: int = 1000,
                         theta: float = 0.05, zeta: float = 10.0, seed=(2, 1),
                         dtype=np.float32) -> np.ndarray:
    """Dominant direction u_b turns by angle theta after every block."""
    rng = rng_for(*seed)
    u = rng.standard_normal(d)
    u /= np.linalg.norm(u)
    out = np.empty((n_blocks * block_rows, d), dtype=np.float64)
    for b in range(n_blocks):
        g = rng.standard_normal(block_rows)
        N = rng.standard_normal((block_rows, d))
        out[b * block_rows:(b + 1) * block_rows] = np.outer(g, u) + N / zeta
        w = rng.standard_normal(d)
        w -= (w @ u) * u
        w /= np.linalg.norm(w)
        u = np.cos(theta) * u + np.sin(theta) * w
        u /= np.linalg.norm(u)
    return out.astype(dtype, copy=False)


def two_subspace_adversarial(n1: int = 5000, n2: int = 5000, d: int = 500,
                             m1: int = 400, m2: int = 4, seed=(9, 0),
                             dtype=np.float64) -> np.ndarray:
    """Rows from coordinates [0, m1), then from [m1, m1+m2); unit norm."""
    rng = rng_for(*seed)
    Y = np.zeros((n1, d))
    Y[:, :m1] = rng.standard_normal((n1, m1))
    Z = np.zeros((n2, d))
    Z[:, m1:m1 + m2] = rng.standard_normal((n2, m2))
    A = np.vstack([Y, Z])
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return A.astype(dtype, copy=False)


def basis_rows(n: int, d: int, seed=(7, 0), dtype=np.float64):
    """Rows c_i e_{j_i}: returns (A, j, c).  Weights are continuous (no ties)."""
    rng = rng_for(*seed)
    p = 1.0 / np.arange(1, d + 1) ** 1.1        # skewed coordinate popularity
    j = rng.choice(d, size=n, p=p / p.sum())
    c = rng.uniform(0.5, 2.0, size=n) * rng.choice([-1.0, 1.0], size=n)
    A = np.zeros((n, d))
    A[np.arange(n), j] = c
    return A.astype(dtype, copy=False), j, c


def batch_shapes(S: int = 512, seed=(4, 0), d_range=(64, 2048), l_range=(16, 128),
                 n_range=(1000, 50_000)):
    """Per-sketch (d, l, n), inclusive uniform integers, drawn d then l then n."""
    rng = rng_for(*seed)
    d = rng.integers(d_range[0], d_range[1] + 1, size=S)
    l = rng.integers(l_range[0], l_range[1] + 1, size=S)
    n = rng.integers(n_range[0], n_range[1] + 1, size=S)
    return d.astype(np.int64), l.astype(np.int64), n.astype(np.int64)


def batch_sketch_rows(i: int, n: int, d: int, l: int, seed=(4, 0), zeta: float = 10.0,
                      dtype=np.float32) -> np.ndarray:
    """Rows of sketch i of the many-sketch workload: Random Noisy with signal
    rank k = max(1, l // 2), drawn from SeedSequence(seed + (i,))."""
    return random_noisy(n, d, max(1, l // 2), zeta, seed=tuple(seed) + (i,), dtype=dtype)


def chunk_sizes(n: int, chunk: int):
    """Row counts of the chunks of an n-row stream (the last one ragged)."""
    return [min(chunk, n - r0) for r0 in range(0, n, chunk)]


def parallel_map(fn, items, workers: int = 16):
    """[fn(x) for x in items] on a thread pool, in order.  NumPy's generators
    and BLAS release the GIL, so independent chunks draw in parallel; every
    chunk has its own seed, so the values do not depend on the pool."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(fn, items))


def random_noisy_device(n: int, d: int, k: int, zeta: float, seed, device="cuda", dtype=None):
    """Random Noisy rows (n x d) drawn on a torch device: the same recipe as
    ``random_noisy`` (D_ii = 1 - (i-1)/k, U orthonormal rows), with S and N
    from a torch.Generator on the device seeded by the key's first 64 bits."""
    import torch
    key = seed if isinstance(seed, (tuple, list)) else (seed,)
    ss = np.random.SeedSequence(list(key))
    g = torch.Generator(device=device)
    g.manual_seed(int(ss.generate_state(1, dtype=np.uint64)[0] & 0x7FFFFFFFFFFFFFFF))
    U = torch.from_numpy(_orthonormal_rows(rng_for(*key, 1), k, d)).to(device)
    D = 1.0 - torch.arange(k, dtype=torch.float64, device=device) / k
    S = torch.randn((n, k), generator=g, dtype=torch.float64, device=device)
    A = (S * D) @ U
    A += torch.randn((n, d), generator=g, dtype=torch.float64, device=device) / zeta
    return A.to(dtype or torch.float32)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even); return raw uint16."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    rounded = rounded.astype(np.uint16)
    rounded[nan] = 0x7FC0
    return rounded


def to_bf16(x: np.ndarray) -> np.ndarray:
    """Values of x rounded to bfloat16, returned as float32 (exactly representable)."""
    b = bf16_bits(x).astype(np.uint32) << 16
    return b.view(np.float32)


# Workload descriptions used by tests and the benchmark.  Sizes follow the
# paper's synthetic recipes scaled to the shapes the sketch is measured on.
WORKLOADS = {
    "c1_random_noisy_10k_x100": dict(n=10_000, d=100, k=10, zeta=10.0, seed=0,
                                     dtype="f64", l=20, variants=("fd",)),
    "c2_random_noisy_100k_x1000": dict(n=100_000, d=1000, k=50, zeta=10.0, seed=(2, 0),
                                       dtype="f32", l=(50, 100, 200),
                                       variants=("fd", "alpha", "fast_alpha", "isvd"),
                                       alpha=0.2),
    "c2_rotating_adversarial_100k_x1000": dict(n=100_000, d=1000, blocks=200, block_rows=500,
                                               theta=0.05, zeta=10.0, seed=(2, 1), dtype="f32",
                                               l=(50, 100, 200)),
    "c3_power_law_200k_x3072": dict(n=200_000, d=3072, r=300, exponent=0.8,
                                    noise_var=1e-2, seed=(3, 0), chunk=50_000, dtype="bf16",
                                    l=256),
    "c4_batch_512": dict(S=512, seed=(4, 0), zeta=10.0, dtype="f32"),
    "c5_random_noisy_1m_x8192": dict(n=1_000_000, d=8192, k=512, zeta=20.0, seed=(5, 0),
                                     chunk=4096, dtype="f32", l=512, alpha=0.2),
}
