"""Oracle results for the workloads at their full sizes (CPU only).

    python tests/golden/make_golden.py c2 | c2_adversarial | c3 | c4 | c5 | eval8192 [--procs N]

Writes ``tests/golden/<name>.json``.  Everything stored comes from the CPU
oracle (``oracle/``) run on rows drawn by the seeded generators
(``paper_1501_06561_amd/synth.py``); nothing here touches the GPU path.  The
GPU tests regenerate the same rows from the same seeds and compare their
sketches with these values: the oracle's covariance error (its own dense
evaluator, Section 1.1), the squared singular values of the oracle's sketch,
Delta, the total shrinkage, ||A||_F^2 and the number of ReduceRank steps.

The oracle takes minutes (c2, c3) to hours (c4, c5) on a CPU, far longer
than a GPU test may run, which is why its results are stored.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1501_06561_amd import synth  # noqa: E402


def _summary(B, st, cov, l):
    """What a GPU sketch is compared against."""
    s = np.linalg.svd(np.asarray(B, dtype=np.float64), compute_uv=False)
    sig2 = np.zeros(l)
    sig2[:min(l, s.size)] = s[:l] ** 2
    return {"cov_err": cov, "sigma2": sig2.tolist(), "fro2B": float(np.sum(sig2)),
            "fro2A": st.fro2A, "Delta": st.Delta, "Stot": st.Stot, "n_rr": st.n_rr,
            "n_rows": st.n_rows}


def _write(name, rec):
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", path, flush=True)


def _sketch(A64, l, variant, alpha=0.2):
    sk = oracle.SketchOracle(A64.shape[1], l, variant, alpha)
    sk.append(A64)
    return sk.finalize(), sk


# --- Random Noisy 100,000 x 1,000, fp32 rows (k = 50, zeta = 10, seed (2, 0))
def c2(_args):
    W = synth.WORKLOADS["c2_random_noisy_100k_x1000"]
    A = synth.random_noisy(W["n"], W["d"], W["k"], W["zeta"], seed=W["seed"], dtype=np.float32)
    A64 = A.astype(np.float64)
    AtA, fa = oracle.gram(A64), oracle.fro2(A64)
    cases = {}
    for variant in W["variants"]:
        for l in W["l"]:
            t = time.time()
            B, st = _sketch(A64, l, variant, W["alpha"])
            cases[f"{variant}_l{l}"] = _summary(B, st, oracle.cov_err_gram(AtA, fa, B), l)
            print(variant, l, cases[f"{variant}_l{l}"]["cov_err"], f"{time.time() - t:.0f}s", flush=True)
    _write("c2_random_noisy_100k_x1000", {"workload": W, "alpha": W["alpha"], "cases": cases})


# --- the slowly rotating adversarial stream, 200 blocks x 500 rows, d = 1,000
def c2_adversarial(_args):
    W = synth.WORKLOADS["c2_rotating_adversarial_100k_x1000"]
    A = synth.rotating_adversarial(W["blocks"], W["block_rows"], W["d"], W["theta"], W["zeta"], seed=W["seed"],
                                   dtype=np.float32)
    A64 = A.astype(np.float64)
    AtA, fa = oracle.gram(A64), oracle.fro2(A64)
    cases = {}
    for variant in ("fd", "isvd", "alpha"):
        for l in W["l"]:
            B, st = _sketch(A64, l, variant, 0.2)
            cases[f"{variant}_l{l}"] = _summary(B, st, oracle.cov_err_gram(AtA, fa, B), l)
            print(variant, l, cases[f"{variant}_l{l}"]["cov_err"], flush=True)
    _write("c2_rotating_adversarial_100k_x1000", {"workload": W, "alpha": 0.2, "cases": cases})


# --- power law, 200,000 x 3,072, bf16 rows, FD l = 256
def c3(_args):
    W = synth.WORKLOADS["c3_power_law_200k_x3072"]
    A = synth.power_law(W["n"], W["d"], r=W["r"], exponent=W["exponent"], noise_var=W["noise_var"],
                        seed=W["seed"], chunk=W["chunk"])
    A64 = synth.to_bf16(A).astype(np.float64)
    del A
    AtA, fa = oracle.gram(A64), oracle.fro2(A64)
    B, st = _sketch(A64, W["l"], "fd")
    rec = _summary(B, st, oracle.cov_err_gram(AtA, fa, B), W["l"])
    print("c3 cov", rec["cov_err"], flush=True)
    _write("c3_power_law_200k_x3072", {"workload": W, "cases": {"fd_l256": rec}})
    # The sketch itself (float32 is ample for a 1e-3 of ||A||_F^2 comparison).
    np.save(os.path.join(HERE, "c3_power_law_200k_x3072_B.npy"), np.asarray(B, dtype=np.float32))


# --- 512 independent sketches of mixed shapes (FD)
def _c4_one(i):
    from threadpoolctl import threadpool_limits
    W = synth.WORKLOADS["c4_batch_512"]
    d, l, n = synth.batch_shapes(W["S"], seed=W["seed"])
    with threadpool_limits(limits=1):
        A = synth.batch_sketch_rows(i, int(n[i]), int(d[i]), int(l[i]))
        A64 = A.astype(np.float64)
        B, st = _sketch(A64, int(l[i]), "fd")
        cov = oracle.cov_err_gram(oracle.gram(A64), oracle.fro2(A64), B)
        rec = _summary(B, st, cov, int(l[i]))
    rec["d"], rec["l"], rec["n"] = int(d[i]), int(l[i]), int(n[i])
    return i, rec


def c4(args):
    W = synth.WORKLOADS["c4_batch_512"]
    out = [None] * W["S"]
    t = time.time()
    with cf.ProcessPoolExecutor(max_workers=args.procs) as ex:
        for done, (i, rec) in enumerate(ex.map(_c4_one, range(W["S"]))):
            out[i] = rec
            if done % 16 == 0:
                print(f"c4 {done + 1}/{W['S']} {time.time() - t:.0f}s", flush=True)
    _write("c4_batch_512", {"workload": W, "sketches": out})


# --- Random Noisy 1,000,000 x 8,192 in 4,096-row chunks, alpha-FD l = 512
def c5(_args):
    W = synth.WORKLOADS["c5_random_noisy_1m_x8192"]
    d, l = W["d"], W["l"]
    U = synth.random_noisy_basis(d, W["k"], tuple(W["seed"]))
    sk = oracle.SketchOracle(d, l, "alpha", W["alpha"])
    AtA = np.zeros((d, d))
    t = time.time()
    for c, rows in enumerate(synth.chunk_sizes(W["n"], W["chunk"])):
        X = synth.random_noisy_chunk(U, rows, W["zeta"], tuple(W["seed"]) + (c + 1,),
                                     dtype=np.float32).astype(np.float64)
        AtA += X.T @ X
        sk.append(X)
        if c % 10 == 0:
            print(f"c5 chunk {c} n_rr {sk.n_rr} {time.time() - t:.0f}s", flush=True)
    B = sk.finalize()
    rec = _summary(B, sk, oracle.cov_err_gram(AtA, sk.fro2A, B), l)
    print("c5 cov", rec["cov_err"], flush=True)
    _write("c5_random_noisy_1m_x8192", {"workload": W, "cases": {"alpha_l512": rec}})
    # The sketch in float16: its entries stay below 2^15 and the rounding
    # (relative 2^-11) moves B^T B by about 1e-5 of ||A||_F^2 here, far inside
    # the 1e-3 bar it is compared at.
    np.save(os.path.join(HERE, "c5_random_noisy_1m_x8192_B.npy"), np.asarray(B, dtype=np.float16))


# --- the evaluator's own check at 8,192 columns: the first chunk of the
# stream above against B = 0.9 times its first 512 rows (any B will do)
def eval8192(_args):
    W = synth.WORKLOADS["c5_random_noisy_1m_x8192"]
    U = synth.random_noisy_basis(W["d"], W["k"], tuple(W["seed"]))
    A = synth.random_noisy_chunk(U, W["chunk"], W["zeta"], tuple(W["seed"]) + (1,), dtype=np.float32)
    A64 = A.astype(np.float64)
    B = 0.9 * A64[:512]
    rec = {"cov_err": oracle.cov_err(A64, B), "fro2A": oracle.fro2(A64),
           "B": "0.9 * rows 0..511 of A", "A": "first 4,096-row chunk of the 1M x 8,192 stream"}
    print(rec, flush=True)
    _write("eval_random_noisy_4096_x8192", rec)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("what", choices=["c2", "c2_adversarial", "c3", "c4", "c5", "eval8192"])
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    globals()[args.what](args)


if __name__ == "__main__":
    main()
