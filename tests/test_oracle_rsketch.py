"""Pins of the hashing and sampling oracle (oracle/rsketch.py) against what
the definitions fix, by routes other than the oracle's own code."""
import numpy as np
import pytest

from oracle import rsketch as R
from paper_1501_06561_amd import synth


def test_splitmix64_reference_outputs():
    """The generator's first outputs from state 0 (the published SplitMix64
    sequence: increment, then the two xor-shift-multiply rounds)."""
    inc = 0x9E3779B97F4A7C15
    assert R.mix(0) == 0xE220A8397B1DCDAF
    assert R.mix(inc) == 0x6E789E6AA1B965F4
    assert R.mix((2 * inc) & ((1 << 64) - 1)) == 0x06C45D188009454F


def test_uniforms_and_buckets_are_in_range_and_roughly_uniform():
    u = np.array([R.uniform(7, i) for i in range(20000)])
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    b = np.array([R.bucket(7, i, 0, 10) for i in range(20000)])
    counts = np.bincount(b, minlength=10)
    assert counts.min() > 1800 and counts.max() < 2200
    s = np.array([R.sign(7, i, 0) for i in range(20000)])
    assert abs(s.mean()) < 0.03


def _dense_S(key, n, l, inst):
    """The projection matrix of Section 2.2 written out: column i has one
    +-1 per stacked instance, scaled by 1/sqrt(instances)."""
    rows = l // inst
    S = np.zeros((l, n))
    for i in range(n):
        for j in range(inst):
            S[j * rows + R.bucket(key, i, j, rows), i] = R.sign(key, i, j) / np.sqrt(inst)
    return S


@pytest.mark.parametrize("kind,l,s", [("hash", 16, 1), ("osnap", 16, 4), ("osnap", 30, 3)])
def test_hashing_equals_the_dense_projection(kind, l, s):
    A = synth.random_noisy(300, 25, 4, 10.0, seed=(30, l))
    B, _ = R.rsketch(A, kind, l, s=s, key=11, chunks=[1, 100, 57])
    S = _dense_S(11, 300, l, 1 if kind == "hash" else s)
    assert np.allclose(B, S @ A, rtol=0, atol=1e-12 * np.abs(A).max() * 300)


def test_hashing_one_row_lands_in_one_bucket():
    a = np.arange(1.0, 6.0)[None, :]
    B, _ = R.rsketch(a, "hash", 8, key=3)
    nz = np.flatnonzero(np.abs(B).sum(axis=1))
    assert nz.size == 1 and np.array_equal(np.abs(B[nz[0]]), a[0])


def test_hashing_is_unbiased_for_the_covariance():
    """E[B^T B] = A^T A over independent keys (each S has E[S^T S] = I)."""
    A = synth.random_noisy(40, 6, 2, 10.0, seed=(31, 0))
    acc = np.zeros((6, 6))
    K = 3000
    for key in range(K):
        B, _ = R.rsketch(A, "osnap", 8, s=2, key=key)
        acc += B.T @ B
    G = A.T @ A
    assert np.max(np.abs(acc / K - G)) <= 0.05 * np.max(np.abs(G))


def test_priority_keeps_everything_when_it_fits():
    A = synth.random_noisy(12, 5, 2, seed=(32, 0))
    B, sk = R.rsketch(A, "priority", 20, key=5, chunks=[3, 4])
    assert sk.tau == 0.0
    assert np.array_equal(B[:12], A) and not B[12:].any()


def test_priority_chunked_equals_the_one_shot_top_l():
    """The streaming reservoir keeps exactly the l rows of largest priority
    over the whole stream, and tau is the (l+1)-th largest priority."""
    A = synth.random_noisy(500, 8, 3, seed=(33, 0))
    _, sk = R.rsketch(A, "priority", 37, key=9, chunks=[1, 50, 200, 3])
    w = np.sum(A * A, axis=1)
    rho = w / np.array([R.uniform(9, i) for i in range(500)])
    top = np.argsort(-rho)[:37]
    assert np.array_equal(np.sort(sk.idx), np.sort(top))
    assert sk.tau == np.sort(rho)[-38]


def test_priority_weights_are_unbiased():
    A = synth.random_noisy(60, 4, 2, seed=(34, 0)) * np.linspace(0.2, 3.0, 60)[:, None]
    fa = np.sum(A * A)
    tot = []
    for key in range(2000):
        _, sk = R.rsketch(A, "priority", 10, key=key, chunks=[13, 22])
        tot.append(np.sum(sk.adjusted_weights()))
    tot = np.array(tot)
    assert abs(tot.mean() - fa) <= 4 * tot.std() / np.sqrt(tot.size)


def _threshold_bisection(w, l):
    lo, hi = 0.0, float(np.sum(w))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.sum(np.minimum(1.0, w / mid)) > l:
            lo = mid
        else:
            hi = mid
    return hi


@pytest.mark.parametrize("chunks", [None, [1, 2, 3, 50], [7] * 40])
def test_varopt_weights_sum_to_the_mass_and_tau_is_the_one_shot_threshold(chunks):
    A = synth.random_noisy(300, 6, 2, seed=(35, 0)) * np.geomspace(0.05, 20.0, 300)[:, None]
    B, sk = R.rsketch(A, "varopt", 25, key=4, chunks=chunks)
    w = np.sum(A * A, axis=1)
    fa = float(np.sum(w))
    assert sk.rows.shape[0] == 25
    assert abs(np.sum(sk.what) - fa) <= 1e-12 * fa
    assert abs(np.sum(B * B) - fa) <= 1e-12 * fa
    tau = _threshold_bisection(w, 25)
    assert abs(sk.tau - tau) <= 1e-12 * tau
    assert set(np.flatnonzero(w >= tau)) <= set(sk.idx.tolist())
    assert np.all(sk.what >= np.minimum(w[sk.idx], tau) * (1 - 1e-12))


def test_varopt_inclusion_probabilities():
    """Row i is kept with probability min(1, w_i / tau) (Monte Carlo over keys)."""
    A = synth.random_noisy(30, 3, 1, seed=(36, 0)) * np.linspace(0.3, 2.5, 30)[:, None]
    w = np.sum(A * A, axis=1)
    tau = _threshold_bisection(w, 8)
    p = np.minimum(1.0, w / tau)
    K = 4000
    hits = np.zeros(30)
    for key in range(K):
        _, sk = R.rsketch(A, "varopt", 8, key=key, chunks=[9, 5, 11])
        hits[sk.idx] += 1
    sd = np.sqrt(np.maximum(p * (1 - p), 1e-12) / K)
    assert np.all(np.abs(hits / K - p) <= 5 * sd + 1e-9)


def test_varopt_keeps_everything_when_it_fits():
    A = synth.random_noisy(9, 4, 2, seed=(37, 0))
    B, sk = R.rsketch(A, "varopt", 9, key=1, chunks=[4])
    assert np.array_equal(B, A)
