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
timed steps), the covariance error of the GPU sketch (device evaluator) and the
CPU oracle timed on the same stream, with the oracle's own covariance error.

`--copy-calibration` instead runs a plain device copy of a known size (the
reference kernel for scaling the FETCH_SIZE / WRITE_SIZE hardware counters).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X FP64 vector and matrix peak, FLOP/s
PEAK_BF16 = 2.5e15       # dense BF16 MFMA, FLOP/s
PEAK_FP8 = 5.0e15        # dense FP8 MFMA, FLOP/s
PEAK_HBM = 8.0e12        # bytes/s
METRIC = "rows/sec sketched at fixed cov-err/||A||_F^2; batched+bf16 vs plain FD, 1 GPU"
CSRC = os.path.join(ROOT, "paper_1501_06561_amd", "csrc")
# Sources that define each stage's kernels; a traffic figure measured with the
# hardware counters is only quoted while these are unchanged.
STAGE_SOURCES = {
    "eig": ["kernels_eig.hip", "fdsk_jacobi.hpp", "fdsk_device.hpp", "fdsk_kernels.hpp"],
    "gram": ["kernels_stream.hip", "fdsk_device.hpp", "fdsk_kernels.hpp"],
    "rebuild": ["kernels_stream.hip", "fdsk_device.hpp", "fdsk_kernels.hpp"],
    "shrink": ["kernels_stream.hip", "fdsk_device.hpp", "fdsk_kernels.hpp"],
    "ingest": ["kernels_stream.hip", "fdsk_device.hpp", "fdsk_kernels.hpp"],
    "tridiag": ["kernels_trid.hip", "fdsk_device.hpp", "fdsk_kernels.hpp"],
    "dc": ["kernels_trid.hip", "fdsk_device.hpp", "fdsk_kernels.hpp"],
    "backtr": ["kernels_trid.hip", "fdsk_device.hpp", "fdsk_kernels.hpp"],
}
KERNELS = {"eig": "k_eig_lds/k_eig_blk (Jacobi)", "gram": "k_gram_f64+k_gram_reduce",
           "rebuild": "k_rebuild_f64", "shrink": "k_shrink", "ingest": "k_ingest",
           "tridiag": "k_tridiag_reg (m <= 208) / k_tridiag", "dc": "k_dc", "backtr": "k_backtr"}


def kernel_name(stage, m):
    """The kernel a stage runs at buffer size m."""
    if stage == "tridiag":
        return "k_tridiag_reg" if m <= 208 else "k_tridiag"
    return KERNELS[stage]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_random_noisy_100k_x1000.json")


def sources_digest(stage):
    h = hashlib.sha256()
    for name in STAGE_SOURCES[stage]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(stage, l, variant):
    """HBM bytes per launch of the stage's kernel from the committed counter
    summary, or None if there is none for this configuration or the kernel
    sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    for e in rec.get("entries", []):
        if e.get("stage") == stage and e.get("l") == l and e.get("variant") == variant:
            if e.get("sources_sha256_16") != sources_digest(stage):
                return None
            return e.get("bytes_per_launch")
    return None


def batched_leg(S, n_max, seq_sketches, seed=(4, 0)):
    """The many-sketch workload (d ~ U{64..2048}, l ~ U{16..128}, n ~
    U{1000..n_max}, Random Noisy rows with k = l/2, zeta = 10, fp32 on the
    device): all sketches through the lock-step batch with FP64 and with
    split-BF16 (x3) Gram/rebuild products, and the first `seq_sketches` of them
    one after another through the single-sketch FP64 path.  Rows/s of each
    (the sequential rate is measured on that prefix of the sketches)."""
    import torch
    from paper_1501_06561_amd import fdsketch, synth
    d, l, n = synth.batch_shapes(S, seed=seed, n_range=(1000, n_max))
    mats = [synth.random_noisy_device(int(n[i]), int(d[i]), max(1, int(l[i]) // 2), 10.0,
                                      (seed[0], seed[1], i)) for i in range(S)]
    rows = int(n.sum())
    # Warm both paths (first launches load the kernels).
    w = fdsketch.FDSketchBatch([dict(d=int(d[i]), l=int(l[i])) for i in range(2)])
    w.append([m[:300] for m in mats[:2]])
    w.finalize()
    w.close()
    torch.cuda.synchronize()
    out = {"workload": f"{S} sketches, d~U{{64..2048}}, l~U{{16..128}}, n~U{{1000..{n_max}}}, "
                       "random noisy k=l/2 zeta=10, fp32 rows on device",
           "rows": rows, "unit": "rows/s"}
    for prec in ("fp64", "bf16x3"):
        b = fdsketch.FDSketchBatch([dict(d=int(d[i]), l=int(l[i]), precision=prec) for i in range(S)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.append(mats)
        b.finalize()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if prec == "fp64":
            out["reduce_steps"] = sum(b.stats(i)["n_reduce"] for i in range(S))
            out["value"] = rows / dt
            out["ms"] = dt * 1e3
        else:
            out["value_bf16x3"] = rows / dt
            out["ms_bf16x3"] = dt * 1e3
        b.close()
    k = min(seq_sketches, S)
    sks = [fdsketch.FDSketch(int(d[i]), int(l[i])) for i in range(k)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sk, m in zip(sks, mats[:k]):
        sk.append(m)
        sk.finalize()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for sk in sks:
        sk.close()
    out["sequential_value"] = int(n[:k].sum()) / t_seq
    out["sequential_sample"] = f"first {k} sketches ({int(n[:k].sum())} rows), single-sketch FP64 path"
    out["speedup_vs_sequential"] = out["value"] / out["sequential_value"]
    out["speedup_bf16x3_vs_sequential"] = out["value_bf16x3"] / out["sequential_value"]
    out["dtype"] = "f64 (bf16x3: split-bf16 Gram/rebuild, f64 eigensolve)"
    return out


def precision_leg(rows, l=256, d=3072, seed=(3, 0)):
    """The power-law workload's shape (d = 3,072, bf16 rows, l = 256, buffer
    512 rows): a prefix of `rows` rows sketched with FP64, BF16, split-BF16
    (x3) and FP8 (x3, Gram only) products.  Per precision: rows/s, the Gram
    and rebuild launches' matrix-core utilisation (their multiply-adds, all
    passes, over the launch time, against the dtype's dense peak) and the
    covariance error's distance from the FP64 sketch's."""
    import numpy as np
    import torch
    from paper_1501_06561_amd import fdsketch, synth
    A = synth.power_law(rows, d, r=300, seed=seed, chunk=rows)
    bits = torch.from_numpy(synth.bf16_bits(A).view(np.int16)).view(torch.bfloat16).cuda()
    m = 2 * l
    keep = l - 1
    npass = {"fp64": 1, "bf16": 1, "bf16x3": 3, "fp8x3": 3}
    peak_gram = {"fp64": PEAK_FP64, "bf16": PEAK_BF16, "bf16x3": PEAK_BF16, "fp8x3": PEAK_FP8}
    peak_rebuild = {"fp64": PEAK_FP64, "bf16": PEAK_BF16, "bf16x3": PEAK_BF16, "fp8x3": PEAK_BF16}
    out = {"workload": f"power-law sigma_i = i^-0.8 over 300 directions + N(0,1e-2), {rows} x {d} "
                       f"bf16 rows, FD l = {l} (buffer {m} rows), "
                       + ("tridiagonal divide-and-conquer" if m <= 512 else "block Jacobi") + " eigensolver",
           "rows": rows}
    cov64 = None
    for prec in ("fp64", "bf16", "bf16x3", "fp8x3"):
        sk = fdsketch.FDSketch(d, l, "fd", precision=prec, profile=True)
        sk.append(bits[:m + 1])                      # warm the kernels
        sk.finalize()
        sk.reset()
        sk.profile()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sk.append(bits)
        sk.finalize()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = sk.profile()
        ev = sk.error(bits, k=10, method=0)
        sk.close()
        g_ms, g_n = prof["gram"]
        r_ms, r_n = prof["rebuild"]
        g_flop = npass[prec] * float(m * (m + 1) * d)
        r_flop = npass[prec] * 2.0 * keep * m * d
        g_tf = g_flop / (g_ms / max(g_n, 1) / 1e3) / 1e12 if g_n else None
        r_tf = r_flop / (r_ms / max(r_n, 1) / 1e3) / 1e12 if r_n else None
        if prec == "fp64":
            cov64 = ev["cov_err"]
        out[prec] = {
            "rows_per_s": rows / dt,
            "gram_us": g_ms / max(g_n, 1) * 1e3, "gram_TFLOPs": g_tf,
            "gram_frac_of_peak": g_tf * 1e12 / peak_gram[prec] if g_tf else None,
            "rebuild_us": r_ms / max(r_n, 1) * 1e3, "rebuild_TFLOPs": r_tf,
            "rebuild_frac_of_peak": r_tf * 1e12 / peak_rebuild[prec] if r_tf else None,
            "eig_ms_per_reduce": prof["eig"][0] / max(prof["eig"][1], 1),
            "cov_err": ev["cov_err"], "abs_diff_vs_fp64": abs(ev["cov_err"] - cov64),
        }
    return out


def host_cpu():
    """The host CPU's model name and logical core count."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": name, "logical_cores": os.cpu_count()}


def copy_calibration(nbytes, reps):
    """A plain device-to-device copy of `nbytes`, `reps` times (counter reference)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
                      "ms_per_copy": dt * 1e3, "GBps_read_plus_write": 2 * nbytes / dt / 1e9}))


def stage_work(stage, m, keep, d, new_rows):
    """Algorithmic work of one launch of a stage: (amount, unit kind, bound)."""
    if stage == "eig":
        return 9.0 * m ** 3, "flop", "alu"          # dense symmetric eigendecomposition
    if stage == "tridiag":
        return 4.0 / 3.0 * m ** 3, "flop", "alu"    # Householder reduction to tridiagonal
    if stage == "dc":
        return 8.0 / 3.0 * m ** 3, "flop", "alu"    # divide-and-conquer products, no deflation
    if stage == "backtr":
        return 2.0 * m ** 3, "flop", "alu"          # m-2 reflectors applied to m vectors
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
    ap.add_argument("--cpu-rows", type=int, default=100_000,
                    help="prefix of the stream the CPU oracle sketches for the baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eig", default="auto", choices=["auto", "jacobi"],
                    help="eigensolver: tridiagonal divide and conquer (m <= 512) or Jacobi")
    ap.add_argument("--rows", type=int, default=100_000,
                    help="rows of the stream to sketch (profiling runs use a prefix)")
    ap.add_argument("--batch-sketches", type=int, default=512,
                    help="sketches in the many-sketch leg (0 skips it)")
    ap.add_argument("--batch-nmax", type=int, default=50_000,
                    help="largest rows per sketch in the many-sketch leg")
    ap.add_argument("--batch-seq", type=int, default=64,
                    help="sketches of the many-sketch leg also run one after another")
    ap.add_argument("--prec-rows", type=int, default=8_000,
                    help="rows of the d = 3,072 precision leg (0 skips it)")
    ap.add_argument("--cpu-1thread-rows", type=int, default=20_000,
                    help="prefix the oracle also sketches with one BLAS thread (0 skips it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter reference) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(args.steps, 1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sketch of one "
              "stream is a sequential chain of ReduceRank steps and this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1501_06561_amd import fdsketch, synth

    N, d, k, zeta, seed = 100_000, 1000, 50, 10.0, (2, 0)
    A = synth.random_noisy(N, d, k, zeta, seed=seed, dtype=np.float32)
    n = max(1, min(args.rows, N))
    A = A[:n]
    At = torch.from_numpy(A).cuda()
    l = args.l
    sk = fdsketch.FDSketch(d, l, args.variant, args.alpha, profile=True, eig=args.eig)
    m = 2 * l

    def step():
        sk.reset()
        sk.append(At)
        return sk.finalize()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sk.profile()                      # drop warmup marks
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_step = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        B = step()                    # finalize synchronises the stream
        per_step.append((time.perf_counter() - ts) * 1e3)
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
    # The dominant kernel: the eigensolve is timed per kernel when it is the
    # tridiagonal route, as one stage when it is a Jacobi solver.
    split = prof["tridiag"][1] > 0
    kernel_stages = [s_ for s_ in prof if prof[s_][1] > 0 and not (split and s_ == "eig")]
    dom = max(kernel_stages, key=lambda s_: prof[s_][0])
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
    roof["traffic"] = measured_traffic(dom, l, args.variant)
    roof["kernel"] = kernel_name(dom, m)
    roof["stage"] = dom
    roof["avg_launch_us"] = avg_s * 1e6
    roof["work_per_launch"] = work

    # Every stage against its own roof.
    kernels = {}
    for s_ in kernel_stages:
        t_ms, nl = prof[s_]
        a_s = t_ms / max(nl, 1) / 1e3
        w, kd, bd = stage_work(s_, m, keep, d, m - keep)
        if kd == "byte":
            kernels[s_] = {"avg_launch_us": a_s * 1e6, "achieved": w / a_s / 1e9, "unit": "GB/s",
                           "peak": PEAK_HBM / 1e9, "frac": w / a_s / PEAK_HBM, "bound": "hbm"}
        else:
            kernels[s_] = {"avg_launch_us": a_s * 1e6, "achieved": w / a_s / 1e12, "unit": "TFLOP/s",
                           "peak": PEAK_FP64 / 1e12, "frac": w / a_s / PEAK_FP64,
                           "bound": "fp64 mfma" if bd == "mfma" else "fp64 alu"}
    # End to end: the time the roofs allow (input bytes at HBM rate, the GEMMs
    # and a 9 m^3 eigendecomposition per ReduceRank at the FP64 peak) over the
    # measured time.
    nrr = st["n_reduce"]              # stats restart with every step (sketch_reset)
    t_bytes = n * d * 4 / PEAK_HBM
    t_gemm = nrr * (m * (m + 1) * d + 2.0 * keep * m * d) / PEAK_FP64
    t_eig = nrr * 9.0 * m ** 3 / PEAK_FP64
    t_min = max(t_bytes, t_gemm, t_eig)
    alg_roof = {"t_min_ms": t_min * 1e3, "t_meas_ms": ms_per_step, "frac": t_min * 1e3 / ms_per_step,
                "terms_ms": {"input_bytes_at_hbm": t_bytes * 1e3, "gemm_at_fp64_peak": t_gemm * 1e3,
                             "eig_9m3_at_fp64_peak": t_eig * 1e3}}

    # Covariance error of the GPU sketch on the device evaluator (untimed).
    ev = sk.error(At, k=10, method=0)
    sk.close()
    del At
    batched = (batched_leg(args.batch_sketches, args.batch_nmax, args.batch_seq)
               if args.batch_sketches > 0 else None)
    prec = precision_leg(args.prec_rows) if args.prec_rows > 0 else None

    cpu = None
    cov_oracle = None
    if not args.no_cpu_baseline:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
        except Exception:
            cores = os.cpu_count()
        rows = min(args.cpu_rows, n)
        A64 = A[:rows].astype(np.float64)
        t = time.perf_counter()
        Bo = oracle.fd_sketch(A64, l, args.variant, args.alpha)
        dt = time.perf_counter() - t
        if rows == n:
            cov_oracle = oracle.cov_err(A64, Bo)
        cpu = {"value": rows / dt, "unit": "rows/s", "cores": cores, "kind": "oracle",
               "sample": (f"first {rows} of the {n} rows of the same stream" if rows < n
                          else f"the whole {n}-row stream") +
                         f", same variant and l (NumPy FP64, LAPACK SVD of the buffer), {dt:.1f} s",
               "host": host_cpu()}
        r1 = min(args.cpu_1thread_rows, n)
        if r1 > 0:
            try:
                from threadpoolctl import threadpool_limits
                with threadpool_limits(limits=1):
                    t = time.perf_counter()
                    oracle.fd_sketch(A[:r1].astype(np.float64), l, args.variant, args.alpha)
                    dt1 = time.perf_counter() - t
                cpu["value_1_thread"] = r1 / dt1
                cpu["sample_1_thread"] = f"first {r1} rows, one BLAS thread, {dt1:.1f} s"
            except Exception as e:      # threadpoolctl missing: report without it
                cpu["value_1_thread"] = None
                cpu["sample_1_thread"] = f"not measured ({type(e).__name__})"

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": float(np.median(per_step)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "random_noisy_100k_x1000_fp32" if n == N else
                   f"random_noisy_100k_x1000_fp32_first_{n}_rows", "n": n, "d": d, "k": k,
                   "zeta": zeta, "variant": args.variant, "l": l, "buffer_rows": m,
                   "alpha": args.alpha if args.variant in ("alpha", "fast_alpha") else None,
                   "eigensolver": "tridiagonal divide and conquer" if split else "Jacobi"},
        "roofline": roof,
        "kernels": kernels,
        "algorithmic_roofline": alg_roof,
        "cpu_baseline": cpu,
        "stages_ms_per_step": {s: prof[s][0] / args.steps for s in prof},
        "batched": batched,
        "precision_leg": prec,
        "cov_err": ev["cov_err"],
        "cov_err_oracle": cov_oracle,
        "reduce_steps": st["n_reduce"],
        "eig_sweeps_avg": st["eig_sweeps"] / max(st["n_reduce"], 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
