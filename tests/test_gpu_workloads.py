"""Parity at the workloads' own shapes on prefixes the oracle finishes inline
(the whole streams are in test_gpu_fullsize.py, against stored results).

* Random Noisy 100,000 x 1,000 fp32 (the single-stream workload): the whole
  stream, FD l = 100, against the oracle on the same rows.
* Power-law 3,072 columns, bf16 rows, l = 256 (buffer 512 rows, the
  tridiagonal route with one pair of launches per column), split-BF16
  Gram/rebuild: the first 20,000 rows of the stream.
* Random Noisy 8,192 columns (rank 512, zeta = 20), alpha-FD with alpha = 0.2,
  l = 512 (buffer 1,024 rows), FP8 Gram: the first 4,096-row chunk of the
  stream.  The oracle's dense evaluator would need an 8,192 x 8,192
  eigendecomposition, so the two sketches are compared through
  ||B_gpu^T B_gpu - B_or^T B_or||_2 / ||A||_F^2, which bounds the difference
  of their covariance errors (triangle inequality), by power iteration on the
  host, and through the device's matrix-free evaluator run on both (pinned at
  8,192 columns in test_gpu_eval.py).
"""
import numpy as np
import pytest

import oracle
from paper_1501_06561_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1501_06561_amd import fdsketch as F  # noqa: E402


def _sketch(A_dev, d, l, variant="fd", alpha=0.2, precision="fp64"):
    sk = F.FDSketch(d, l, variant, alpha, precision=precision)
    sk.append(A_dev)
    B = sk.finalize().cpu().numpy()
    st = sk.stats()
    return sk, B, st


def _gram_diff_norm(B1, B2, iters=200, seed=0):
    """||B1^T B1 - B2^T B2||_2 by power iteration (symmetric operator)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(B1.shape[1])
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = B1.T @ (B1 @ x) - B2.T @ (B2 @ x)
        lam_new = np.linalg.norm(y)
        if lam_new == 0.0:
            return 0.0
        x = y / lam_new
        if abs(lam_new - lam) <= 1e-10 * lam_new:
            break
        lam = lam_new
    return lam_new


def test_random_noisy_100k_x1000_fd_l100_whole_stream():
    A = synth.random_noisy(100_000, 1000, 50, 10.0, seed=(2, 0), dtype=np.float32)
    sk, B, st = _sketch(torch.from_numpy(A).cuda(), 1000, 100)
    A64 = A.astype(np.float64)
    Bo, so = oracle.fd_sketch(A64, 100, "fd", return_state=True)
    ce, co = oracle.cov_err(A64, B), oracle.cov_err(A64, Bo)
    assert abs(ce - co) <= 1e-6 * co, (ce, co)
    assert st["n_reduce"] == so.n_rr == 990
    fa = oracle.fro2(A64)
    assert abs(st["fro2_A"] - fa) <= 1e-12 * fa
    assert abs(fa - oracle.fro2(B) - st["shrink_total"]) <= 1e-9 * fa
    # The device evaluator on the full stream agrees with the oracle's.
    ev = sk.error(torch.from_numpy(A).cuda())
    assert abs(ev["cov_err"] - ce) <= 1e-9 * ce
    sk.close()


def test_power_law_3072_bf16_l256_prefix_bf16x3():
    A = synth.power_law(50_000, 3072, r=300, seed=(3, 0))[:20_000]
    Ab = synth.to_bf16(A).astype(np.float64)
    bits = torch.from_numpy(synth.bf16_bits(A).view(np.int16)).view(torch.bfloat16).cuda()
    sk, B, st = _sketch(bits, 3072, 256, precision="bf16x3")
    Bo, so = oracle.fd_sketch(Ab, 256, "fd", return_state=True)
    ce, co = oracle.cov_err(Ab, B), oracle.cov_err(Ab, Bo)
    assert abs(ce - co) <= 1e-4, (ce, co)
    assert st["n_reduce"] == so.n_rr
    assert st["eig_unconverged"] == 0
    sk.close()


def test_random_noisy_8192_alpha_l512_first_chunk_fp8x3():
    d, k, l = 8192, 512, 512
    U = synth.random_noisy_basis(d, k, (5, 0))
    A = synth.random_noisy_chunk(U, 4096, 20.0, (5, 0, 1), dtype=np.float32)
    sk, B, st = _sketch(torch.from_numpy(A).cuda(), d, l, "alpha", 0.2, precision="fp8x3")
    A64 = A.astype(np.float64)
    Bo, so = oracle.fd_sketch(A64, l, "alpha", 0.2, return_state=True)
    fa = oracle.fro2(A64)
    assert st["n_reduce"] == so.n_rr
    assert _gram_diff_norm(B, Bo) / fa <= 1e-3
    # The same matrix-free device evaluator on both sketches (the evaluator
    # is checked against the oracle's at smaller sizes in test_gpu_eval.py).
    Ad = torch.from_numpy(A).cuda()
    ce = F.evaluate(Ad, torch.from_numpy(B).cuda(), method=1)["cov_err"]
    co = F.evaluate(Ad, torch.from_numpy(Bo).cuda(), method=1)["cov_err"]
    assert abs(ce - co) <= 1e-3, (ce, co)
    assert st["eig_unconverged"] == 0
    sk.close()
