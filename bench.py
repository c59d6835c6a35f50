#!/usr/bin/env python
"""Rows/s sketched by the Frequent Directions hot path on one MI355X.

Workload: the "Random Noisy" construction of the paper's Section 4 at
100,000 x 1,000 (signal rank k = 50, zeta = 10, seed (2, 0)), rows stored as
fp32 and already resident in HBM.  One step = one whole pass of the hot path
over every row: ingest, every scheduled ReduceRank (Gram, eigensolve, shrink,
rebuild) and finalize, for the chosen variant and sketch size (default: FD,
l = 100, buffer 2l = 200 rows).  Arithmetic is FP64.

Prints one JSON line with the metric, the dominant kernel's roofline (stage
times come from HIP events the library records on its stream during the
timed steps) and the CPU oracle timed on a bounded prefix of the same stream.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X FP64 vector and matrix peak, FLOP/s
PEAK_HBM = 8.0e12        # bytes/s


def stage_work(stage, m, keep, d, new_rows):
    """Algorithmic work of one launch of a stage: (amount, unit kind, bound)."""
    if stage == "eig":
        return 9.0 * m ** 3, "flop", "alu"          # dense symmetric eigendecomposition
    if stage == "gram":
        return float(m * (m + 1) * d), "flop", "mfma"   # symmetric m x m x d
    if stage == "rebuild":
        return 2.0 * keep * m * d, "flop", "mfma"
    if stage == "ingest":
        return float(new_rows * d * (4 + 8)), "byte", "hbm"   # fp32 in, fp64 buffer out
    return 0.0, "flop", "alu"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variant", default="fd", choices=["fd", "isvd", "alpha", "fast_alpha"])
    ap.add_argument("--l", type=int, default=100)
    ap.add_argument("--alpha", type=float, default=0.2)
    ap.add_argument("--cpu-rows", type=int, default=20_000,
                    help="prefix of the stream the CPU oracle sketches for the baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sketch of one "
              "stream is a sequential chain of ReduceRank steps and this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1501_06561_amd import fdsketch, synth

    n, d, k, zeta, seed = 100_000, 1000, 50, 10.0, (2, 0)
    A = synth.random_noisy(n, d, k, zeta, seed=seed, dtype=np.float32)
    At = torch.from_numpy(A).cuda()
    l = args.l
    sk = fdsketch.FDSketch(d, l, args.variant, args.alpha, profile=True)
    m = 2 * l

    def step():
        sk.reset()
        sk.append(At)
        return sk.finalize()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sk.profile()                      # drop warmup marks
    stats_before = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sk.profile()
    st = sk.stats()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3)

    # Dominant stage and its roofline.
    keep = {"fd": l - 1, "isvd": l - 1, "alpha": l - 1}.get(args.variant)
    if keep is None:
        s_ = int(np.ceil(args.alpha * l * (1 - 1e-12)))
        keep = (l - s_) + (s_ + 1) // 2 - 1
    dom = max(prof, key=lambda s: prof[s][0])
    tot_ms, launches = prof[dom]
    avg_s = tot_ms / max(launches, 1) / 1e3
    work, kind, bound = stage_work(dom, m, keep, d, m - keep)
    if kind == "byte":
        roof = {"bound": "hbm", "achieved": work / avg_s / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s"}
    else:
        roof = {"bound": bound, "achieved": work / avg_s / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = {"eig": "k_eig_lds/k_eig_blk", "gram": "k_gram_f64+k_gram_reduce",
                      "rebuild": "k_rebuild_f64", "shrink": "k_shrink", "ingest": "k_ingest"}[dom]
    roof["stage"] = dom
    roof["avg_launch_us"] = avg_s * 1e6
    roof["work_per_launch"] = work

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
        except Exception:
            cores = os.cpu_count()
        rows = min(args.cpu_rows, n)
        t = time.perf_counter()
        oracle.fd_sketch(A[:rows].astype(np.float64), l, args.variant, args.alpha)
        dt = time.perf_counter() - t
        cpu = {"value": rows / dt, "unit": "rows/s", "cores": cores, "kind": "oracle",
               "sample": f"first {rows} rows of the same stream, same variant and l "
                         f"(NumPy FP64, LAPACK SVD of the buffer), {dt:.1f} s"}

    out = {
        "metric": "rows/sec sketched at fixed cov-err/||A||_F^2 (FP64-faithful FD path)",
        "value": value,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random_noisy_100k_x1000_fp32", "n": n, "d": d, "k": k,
                   "zeta": zeta, "variant": args.variant, "l": l, "buffer_rows": m,
                   "alpha": args.alpha if args.variant in ("alpha", "fast_alpha") else None},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms_per_step": {s: prof[s][0] / args.steps for s in prof},
        "reduce_steps": st["n_reduce"],
        "eig_sweeps_avg": st["eig_sweeps"] / max(st["n_reduce"], 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
