#!/usr/bin/env python
"""Rows/s sketched by the Frequent Directions hot path on one MI355X.

Headline workload: 512 independent sketches of mixed shapes (d ~ U{64..2048},
l ~ U{16..128}, n ~ U{1000..50000}; each stream the Random Noisy construction
of the paper's Section 4 with signal rank k = l/2 and zeta = 10, fp32 rows
resident in HBM; 13.2 million rows in all), Frequent Directions (Algorithm 1,
buffer 2l).  One step = the whole hot path over every row of every sketch:
ingest, every scheduled ReduceRank (Gram, eigensolve, shrink, rebuild) and
finalize, through the batch (each size class of buffer rows on a stream of
its own, one launch per stage and round) with split-BF16 (x3) Gram and
rebuild products and the FP64 eigensolve, shrink and accumulators.  The same
step replayed from HIP graphs captured per size class is timed beside it.  Beside it, on the same rows: the same batch in FP64, and plain
FP64 FD run one sketch after another (the single-sketch path).  After the
timed steps every sketch's covariance error (device evaluator) is checked
against the oracle's stored result for that sketch.

Extra legs: FD l = 100 on the Random Noisy 100,000 x 1,000 stream (single
sketch, per-stage times), and the d = 3,072 shape of the power-law workload
with each product precision (matrix-core rates).

Prints one JSON line.  `--copy-calibration BYTES` instead runs a plain device
copy of a known size (the reference for scaling FETCH_SIZE / WRITE_SIZE).
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
GOLDEN = os.path.join(ROOT, "tests", "golden")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batch_512.json")

# Kernels behind each profiled stage and the sources that define them (a
# counter-measured traffic figure is quoted only while these are unchanged).
STAGE_KERNELS = {
    "ingest": ("kg_ingest", ["kernels_stream.hip"]),
    "gram": ("kg_split_bf16+kg_gram_bf16<3>+kg_mirror (fp64: kg_gram)", ["kernels_lowp.hip", "kernels_stream.hip"]),
    "tridiag_head": ("kg_tridiag", ["kernels_trid.hip"]),
    "tridiag": ("kg_tridiag_reg", ["kernels_trid.hip"]),
    "dc": ("kg_dc", ["kernels_trid.hip"]),
    "backtr": ("kg_backtr", ["kernels_trid.hip"]),
    "shrink": ("kg_shrink", ["kernels_stream.hip"]),
    "rebuild": ("kg_rebuild_bf16<3> (fp64: kg_rebuild)", ["kernels_lowp.hip", "kernels_stream.hip"]),
}
COMMON_SOURCES = ["fdsk_device.hpp", "fdsk_kernels.hpp", "fdsk_batch.hpp"]


def sources_digest(stage):
    h = hashlib.sha256()
    for name in STAGE_KERNELS[stage][1] + COMMON_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(stage):
    """HBM bytes per launch of the stage's kernel from the committed counter
    summary, or None when there is none or the kernel's sources changed."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    e = rec.get("stages", {}).get(stage)
    if not e or e.get("sources_sha256_16") != sources_digest(stage):
        return None
    return e.get("bytes_per_launch")


def host_cpu():
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


def stage_table(prof, peak_of):
    """Every profiled stage against its own roof: {stage: {...}}."""
    out = {}
    for name, (ms, launches, work) in prof.items():
        if launches == 0:
            continue
        secs = ms / 1e3
        if name == "ingest":
            ach, unit, peak, bound = work / secs / 1e9, "GB/s", PEAK_HBM / 1e9, "hbm"
        else:
            pk, bound = peak_of(name)
            ach, unit, peak = work / secs / 1e12, "TFLOP/s", pk / 1e12
        out[name] = {"ms": ms, "launches": launches, "avg_launch_us": ms / launches * 1e3,
                     "work_per_launch": work / launches, "achieved": ach, "unit": unit, "peak": peak,
                     "frac": ach / peak if peak else None, "bound": bound}
    return out


def make_batch_rows(S, seed):
    """The 512-sketch workload's rows, drawn by the seeded generator on the
    host (16 threads) and moved to the device as fp32."""
    import numpy as np
    import torch
    from paper_1501_06561_amd import synth
    d, l, n = synth.batch_shapes(S, seed=seed)

    def one(i):
        return torch.from_numpy(synth.batch_sketch_rows(i, int(n[i]), int(d[i]), int(l[i]), seed=seed)).cuda()
    rows = synth.parallel_map(one, range(S), workers=16)
    torch.cuda.synchronize()
    return np.asarray(d), np.asarray(l), np.asarray(n), rows


def batch_parity(rows, outs, l, precision, golden):
    """Per-sketch covariance error of the GPU sketches (device evaluator)
    against the oracle's stored value for the same sketch."""
    from paper_1501_06561_amd import fdsketch as F
    worst_abs, worst_rel, bad = 0.0, 0.0, []
    for i, (A, B) in enumerate(zip(rows, outs)):
        ce = F.evaluate(A, B, k=10, method=0)["cov_err"]
        co = golden[i]["cov_err"]
        diff = abs(ce - co)
        worst_abs = max(worst_abs, diff)
        worst_rel = max(worst_rel, diff / co if co > 0 else 0.0)
        ok = diff <= (1e-6 * co + 1e-12 if precision == "fp64" else 1e-3)
        if not ok:
            bad.append(i)
    bar = "|cov_gpu - cov_oracle| <= 1e-6 cov_oracle + 1e-12" if precision == "fp64" else \
        "|cov_gpu - cov_oracle| <= 1e-3"
    return {"sketches": len(outs), "failed": bad, "max_abs_diff": worst_abs, "max_rel_diff": worst_rel,
            "bar": bar, "ok": not bad}


def run_batch(cfgs, rows, steps, warmup, profile=False, graph=False):
    """Steps of reset + append + finalize on one batch: (ms per step, per-step
    ms, outputs of the last step, batch)."""
    import torch
    from paper_1501_06561_amd import fdsketch as F
    b = F.FDSketchBatch(cfgs, profile=profile, graph=graph)
    outs = None
    for _ in range(warmup):
        b.reset()
        b.append(rows)
        outs = b.finalize()
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        b.reset()
        b.append(rows)
        outs = b.finalize()            # synchronises the batch's stream
        per.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    return ms, per, outs, b


def sequential_leg(d, l, rows, k):
    """Plain FP64 FD, the first k sketches one after another through the
    single-sketch path (sketches created beforehand, as the batch is)."""
    import torch
    from paper_1501_06561_amd import fdsketch as F
    sks = [F.FDSketch(int(d[i]), int(l[i])) for i in range(k)]
    # Warm every kernel shape once (first launches load code objects).
    for sk, A in zip(sks[:8], rows[:8]):
        sk.append(A[: 2 * sk.l + 1])
        sk.finalize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for sk, A in zip(sks, rows[:k]):
        sk.reset()
        sk.append(A)
        outs.append(sk.finalize())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for sk in sks:
        sk.close()
    return dt, outs


def single_stream_leg(l=100):
    """FD on the Random Noisy 100,000 x 1,000 fp32 stream (k = 50, zeta = 10,
    seed (2, 0)) through the single-sketch path: rows/s and per-stage times."""
    import numpy as np
    import torch
    from paper_1501_06561_amd import fdsketch as F, synth
    W = synth.WORKLOADS["c2_random_noisy_100k_x1000"]
    A = synth.random_noisy(W["n"], W["d"], W["k"], W["zeta"], seed=W["seed"], dtype=np.float32)
    At = torch.from_numpy(A).cuda()
    sk = F.FDSketch(W["d"], l, "fd", profile=True)
    sk.append(At)
    sk.finalize()
    sk.reset()
    sk.profile()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sk.append(At)
    B = sk.finalize()
    dt = time.perf_counter() - t0
    prof = sk.profile()
    st = sk.stats()
    ev = sk.error(At, k=10, method=0)
    sk.close()
    table = stage_table(prof, lambda s_: (PEAK_FP64, "fp64 mfma" if s_ in ("gram", "rebuild") else "fp64 alu"))
    return {"workload": "random_noisy_100k_x1000_fp32, FD l = 100 (buffer 200 rows), FP64",
            "rows_per_s": W["n"] / dt, "ms": dt * 1e3, "reduce_steps": st["n_reduce"],
            "cov_err": ev["cov_err"], "stages": table,
            "eig_ms_per_reduce": prof["eig"][0] / max(prof["eig"][1], 1)}, A, B


def precision_leg(rows, l=256, d=3072, seed=(3, 0)):
    """The power-law workload's shape (d = 3,072, bf16 rows, l = 256, buffer
    512 rows): a prefix of `rows` rows sketched with FP64, split-BF16 (x3) and
    FP8 (x3, Gram only) products.  Per precision: rows/s, the Gram and
    rebuild launches' rate (their multiply-adds, all passes, over the launch
    time, against the dtype's dense peak) and the covariance error's distance
    from the FP64 sketch's."""
    import numpy as np
    import torch
    from paper_1501_06561_amd import fdsketch as F, synth
    A = synth.power_law(rows, d, r=300, seed=seed, chunk=rows)
    bits = torch.from_numpy(synth.bf16_bits(A).view(np.int16)).view(torch.bfloat16).cuda()
    m = 2 * l
    peak_gram = {"fp64": PEAK_FP64, "bf16x3": PEAK_BF16, "fp8x3": PEAK_FP8}
    peak_rebuild = {"fp64": PEAK_FP64, "bf16x3": PEAK_BF16, "fp8x3": PEAK_BF16}
    out = {"workload": f"power-law sigma_i = i^-0.8 over 300 directions + N(0,1e-2), {rows} x {d} "
                       f"bf16 rows, FD l = {l} (buffer {m} rows)", "rows": rows}
    cov64 = None
    for prec in ("fp64", "bf16x3", "fp8x3"):
        sk = F.FDSketch(d, l, "fd", precision=prec, profile=True)
        sk.append(bits[:m + 1])
        sk.finalize()
        sk.reset()
        sk.profile()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sk.append(bits)
        sk.finalize()
        dt = time.perf_counter() - t0
        prof = sk.profile()
        ev = sk.error(bits, k=10, method=0)
        sk.close()
        if prec == "fp64":
            cov64 = ev["cov_err"]
        g_ms, g_n, g_w = prof["gram"]
        r_ms, r_n, r_w = prof["rebuild"]
        out[prec] = {
            "rows_per_s": rows / dt,
            "gram_us": g_ms / max(g_n, 1) * 1e3, "gram_TFLOPs": g_w / (g_ms / 1e3) / 1e12,
            "gram_frac_of_peak": g_w / (g_ms / 1e3) / peak_gram[prec],
            "rebuild_us": r_ms / max(r_n, 1) * 1e3, "rebuild_TFLOPs": r_w / (r_ms / 1e3) / 1e12,
            "rebuild_frac_of_peak": r_w / (r_ms / 1e3) / peak_rebuild[prec],
            "eig_ms_per_reduce": prof["eig"][0] / max(prof["eig"][1], 1),
            "cov_err": ev["cov_err"], "abs_diff_vs_fp64": abs(ev["cov_err"] - cov64),
        }
    return out


def rsketch_leg(A, reps=10, l=1000):
    """The hashing and sampling sketches (Sections 2.2 and 3.2) over the
    Random Noisy 100,000 x 1,000 fp32 block appended `reps` times (one append
    call per block): rows/s, the HBM rate of the row reads (n d 4 bytes)
    against 8 TB/s, and each sketch's covariance error over the whole stream
    (device evaluator)."""
    import torch
    from paper_1501_06561_amd import fdsketch as F
    At = A if A.is_cuda else A.cuda()
    n1, d = At.shape
    out = {"workload": f"random_noisy_100k_x1000_fp32 appended {reps} times ({n1 * reps} rows), l = {l}, "
                       "OSNAP s = 4", "bytes_per_row": d * 4}
    full = At.repeat(reps, 1)
    for kind in ("hash", "osnap", "priority", "varopt"):
        sk = F.RSketch(kind, d, l, s=4, key=1)
        sk.append(At[: 2 * l])              # first launches load the kernels
        sk.close()
        sk = F.RSketch(kind, d, l, s=4, key=1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            sk.append(At)
        e1.record()
        B, _ = sk.finalize()
        ms = e0.elapsed_time(e1)
        sk.close()
        rows = n1 * reps
        ev = F.evaluate(full, B, k=10, method=0)
        out[kind] = {"rows_per_s": rows / (ms / 1e3), "ms": ms,
                     "read_GBps": rows * d * 4 / (ms / 1e3) / 1e9,
                     "frac_of_hbm": rows * d * 4 / (ms / 1e3) / PEAK_HBM, "cov_err": ev["cov_err"]}
    del full
    return out


def large_stream_leg(rows_limit=None):
    """alpha-FD (alpha = 0.2, l = 512, buffer 1,024 rows) over the Random
    Noisy 1,000,000 x 8,192 stream (rank 512, zeta = 20), fp32 rows resident
    in HBM and appended in 4,096-row chunks, FP8 Gram with split
    compensation: rows/s and per-stage times."""
    import torch
    from paper_1501_06561_amd import fdsketch as F, synth
    W = synth.WORKLOADS["c5_random_noisy_1m_x8192"]
    d, l = W["d"], W["l"]
    U = synth.random_noisy_basis(d, W["k"], tuple(W["seed"]))
    sizes = synth.chunk_sizes(W["n"] if rows_limit is None else rows_limit, W["chunk"])
    n = sum(sizes)
    A = torch.empty((n, d), dtype=torch.float32, device="cuda")
    r0 = 0
    for g0 in range(0, len(sizes), 16):
        grp = list(range(g0, min(g0 + 16, len(sizes))))
        chunks = synth.parallel_map(
            lambda c: synth.random_noisy_chunk(U, sizes[c], W["zeta"], tuple(W["seed"]) + (c + 1,)), grp, 16)
        for X in chunks:
            A[r0:r0 + X.shape[0]].copy_(torch.from_numpy(X))
            r0 += X.shape[0]
    sk = F.FDSketch(d, l, "alpha", W["alpha"], precision="fp8x3", profile=True)
    sk.append(A[: 2 * l + 1])
    sk.finalize()
    sk.reset()
    sk.profile()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0 = 0
    for c in sizes:
        sk.append(A[r0:r0 + c])
        r0 += c
    sk.finalize()
    dt = time.perf_counter() - t0
    prof = sk.profile()
    st = sk.stats()
    sk.close()
    del A
    table = stage_table({k_: v for k_, v in prof.items() if k_ != "eig"},
                        lambda s_: ((PEAK_FP8, "fp8 mfma") if s_ == "gram" else (PEAK_BF16, "bf16 mfma")
                                    if s_ == "rebuild" else (PEAK_FP64, "fp64 alu")))
    return {"workload": f"random_noisy_1m_x8192_fp32 ({n} rows in 4,096-row chunks), alpha-FD alpha = 0.2, "
                        "l = 512 (buffer 1,024 rows), FP8x3 Gram, split-BF16 rebuild, FP64 eigensolve",
            "rows_per_s": n / dt, "s": dt, "reduce_steps": st["n_reduce"],
            "eig_ms_per_reduce": prof["eig"][0] / max(prof["eig"][1], 1), "stages": table}


def gram_only_leg(reps=20):
    """Only the Gram products (fdsk_gram) at the buffer shapes of the
    reduced-precision workloads, for hardware-counter runs: FP64 and
    split-BF16 x3 on 512 x 3,072, FP8 x3 on 1,024 x 8,192."""
    import numpy as np
    import torch
    from paper_1501_06561_amd import fdsketch as F, synth
    out = {}
    for name, m, d, prec in (("fp64_512x3072", 512, 3072, "fp64"), ("bf16x3_512x3072", 512, 3072, "bf16x3"),
                             ("fp8x3_1024x8192", 1024, 8192, "fp8x3")):
        C = torch.from_numpy(synth.random_noisy(m, d, m // 4, 10.0, seed=(8, m))).cuda()
        F.gram(C, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            F.gram(C, prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        out[name] = {"ms_per_call": ms, "calls": reps, "flops_per_call": (1 if prec == "fp64" else 3) * m * (m + 1) * d}
    return out


def cpu_baseline_leg(d, l, n, seed, seconds):
    """The oracle (NumPy FP64, LAPACK SVD of the buffer) on the first
    sketches of the same workload until about `seconds` of CPU work."""
    import numpy as np
    import oracle
    from paper_1501_06561_amd import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
    except Exception:
        cores = os.cpu_count()
    done_rows, spent, k = 0, 0.0, 0
    while spent < seconds and k < len(n):
        A = synth.batch_sketch_rows(k, int(n[k]), int(d[k]), int(l[k]), seed=seed).astype(np.float64)
        t = time.perf_counter()
        oracle.fd_sketch(A, int(l[k]))
        spent += time.perf_counter() - t
        done_rows += int(n[k])
        k += 1
    return {"value": done_rows / spent, "unit": "rows/s", "cores": cores, "kind": "oracle",
            "sample": f"the first {k} of the 512 sketches ({done_rows} rows), FD at each sketch's l, "
                      f"NumPy FP64 with LAPACK's SVD of the buffer, {spent:.1f} s",
            "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seq", type=int, default=512,
                    help="sketches of the plain FP64 one-after-another leg (0 skips it)")
    ap.add_argument("--no-parity", action="store_true", help="skip the per-sketch oracle check")
    ap.add_argument("--graph", action="store_true",
                    help="headline through per-class HIP graphs instead of direct launches")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the single-stream and precision legs")
    ap.add_argument("--prec-rows", type=int, default=8_000)
    ap.add_argument("--precision-only", action="store_true",
                    help="only the precision leg (for matrix-core counter runs)")
    ap.add_argument("--large-stream", action="store_true",
                    help="only the 1,000,000 x 8,192 alpha-FD stream (FP8 Gram), about a minute")
    ap.add_argument("--single-only", action="store_true",
                    help="only the single-sketch FD l = 100 leg on the 100,000 x 1,000 stream "
                         "(for hardware-counter runs)")
    ap.add_argument("--prec-l", type=int, default=256)
    ap.add_argument("--prec-d", type=int, default=3072)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-only", action="store_true",
                    help="one warm-up and one step of the split-BF16 batch, nothing else "
                         "(for hardware-counter runs)")
    ap.add_argument("--gram-only", action="store_true",
                    help="only the Gram products at the reduced-precision buffer shapes (for counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter reference) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(args.steps, 1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the batch is sharded "
              "across GPUs only by design (independent sketches), not in this build.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1501_06561_amd import synth

    if args.gram_only:
        print(json.dumps({"gram_only": gram_only_leg()}))
        return
    if args.precision_only:
        print(json.dumps({"precision_leg": precision_leg(args.prec_rows, l=args.prec_l, d=args.prec_d)}))
        return
    if args.single_only:
        print(json.dumps({"single_stream": single_stream_leg()[0]}))
        return
    if args.large_stream:
        print(json.dumps({"large_stream": large_stream_leg()}))
        return

    W = synth.WORKLOADS["c4_batch_512"]
    S, seed = W["S"], tuple(W["seed"])
    t_gen = time.perf_counter()
    d, l, n, rows = make_batch_rows(S, seed)
    t_gen = time.perf_counter() - t_gen
    total_rows = int(n.sum())
    cfg = lambda prec: [dict(d=int(d[i]), l=int(l[i]), precision=prec) for i in range(S)]
    graph = args.graph
    print(f"[bench] rows drawn and resident: {total_rows} rows in {t_gen:.1f} s", file=sys.stderr, flush=True)

    if args.profile_only:
        ms, per, outs, b = run_batch(cfg("bf16x3"), rows, 1, 1, graph=graph)
        b.close()
        print(json.dumps({"profile_only": True, "ms": ms, "rows": total_rows}))
        return

    # Headline: the split-BF16 batch.
    ms, per, outs_bf, b = run_batch(cfg("bf16x3"), rows, args.steps, args.warmup, graph=graph)
    st_bf = [b.stats(i) for i in range(S)]
    b.close()
    value = total_rows / (ms / 1e3)
    print(f"[bench] batch bf16x3: {ms:.1f} ms/step, {value:.4g} rows/s", file=sys.stderr, flush=True)

    # The same batch with the launch-shape tuner off (fixed default shapes).
    from paper_1501_06561_amd import fdsketch as F
    mode = F.tune_mode()
    F.tune_mode("off")
    ms_fixed, _, _, b = run_batch(cfg("bf16x3"), rows, 1, 1, graph=graph)
    b.close()
    F.tune_mode(mode)
    tuning = {"mode": mode, "cache": F.tune_path(), "fixed_shapes_ms_per_step": ms_fixed,
              "choices": {k_: {"value": v_[0], "timings_us": v_[1]} for k_, v_ in F.tune_table().items()}}
    print(f"[bench] batch bf16x3, fixed shapes: {ms_fixed:.1f} ms/step", file=sys.stderr, flush=True)

    # The same batch in FP64.
    ms64, per64, outs_64, b = run_batch(cfg("fp64"), rows, 1, 1, graph=graph)
    b.close()
    print(f"[bench] batch fp64: {ms64:.1f} ms", file=sys.stderr, flush=True)
    # The other launch mode of the split-BF16 batch (graph replay or direct).
    ms_alt, per_alt, _, b = run_batch(cfg("bf16x3"), rows, 1, 1, graph=not graph)
    b.close()
    print(f"[bench] batch bf16x3 {'direct' if graph else 'graph'}: {ms_alt:.1f} ms", file=sys.stderr,
          flush=True)

    # One profiled step of each precision: per-stage times on the class streams.
    ms_p, _, _, bp = run_batch(cfg("bf16x3"), rows, 1, 0, profile=True)
    prof_bf = bp.profile()
    bp.close()
    ms_p64, _, _, bp = run_batch(cfg("fp64"), rows, 1, 0, profile=True)
    prof_64 = bp.profile()
    bp.close()
    peak_bf = lambda s_: ((PEAK_BF16, "bf16 mfma") if s_ in ("gram", "rebuild") else (PEAK_FP64, "fp64 alu"))
    peak_64 = lambda s_: ((PEAK_FP64, "fp64 mfma") if s_ in ("gram", "rebuild") else (PEAK_FP64, "fp64 alu"))
    stages_bf = stage_table({k_: v for k_, v in prof_bf.items() if k_ != "eig"}, peak_bf)
    stages_64 = stage_table({k_: v for k_, v in prof_64.items() if k_ != "eig"}, peak_64)
    dom = max(stages_bf, key=lambda s_: stages_bf[s_]["ms"])
    e = stages_bf[dom]
    roof = {"bound": "hbm" if e["bound"] == "hbm" else ("mfma" if "mfma" in e["bound"] else "alu"),
            "achieved": e["achieved"], "peak": e["peak"], "unit": e["unit"], "frac": e["frac"],
            "traffic": measured_traffic(dom), "kernel": STAGE_KERNELS[dom][0], "stage": dom,
            "avg_launch_us": e["avg_launch_us"], "work_per_launch": e["work_per_launch"],
            "launches": e["launches"],
            "note": "a launch serves every sketch of its round and size class; achieved = the "
                    "algorithmic flops of those sketches / the launch time (HIP events on the class "
                    "stream, one profiled step of the same batch)"}

    # Plain FP64 FD, one sketch after another.
    seq = None
    if args.seq > 0:
        k = min(args.seq, S)
        dt_seq, outs_seq = sequential_leg(d, l, rows, k)
        seq_rows = int(n[:k].sum())
        seq = {"value": seq_rows / dt_seq, "unit": "rows/s", "ms": dt_seq * 1e3, "sketches": k,
               "rows": seq_rows, "path": "single-sketch FP64 path, sketches one after another"}
        print(f"[bench] sequential fp64: {dt_seq:.1f} s", file=sys.stderr, flush=True)

    # Parity of every sketch against the oracle's stored result.
    parity = None
    gpath = os.path.join(GOLDEN, "c4_batch_512.json")
    if not args.no_parity and os.path.exists(gpath):
        with open(gpath) as f:
            gold = json.load(f)["sketches"]
        parity = {"bf16x3": batch_parity(rows, outs_bf, l, "bf16x3", gold),
                  "fp64": batch_parity(rows, outs_64, l, "fp64", gold)}
        if seq is not None and seq["sketches"] == S:
            parity["sequential_fp64"] = batch_parity(rows, outs_seq, l, "fp64", gold)
    elif not args.no_parity:
        parity = {"skipped": "no stored oracle results (tests/golden/c4_batch_512.json)"}
    print("[bench] parity done", file=sys.stderr, flush=True)
    del outs_bf, outs_64
    if seq is not None:
        del outs_seq

    extra_single = extra_prec = extra_rs = None
    if not args.no_extra:
        extra_single, A_c2, _ = single_stream_leg()
        print("[bench] single stream done", file=sys.stderr, flush=True)
        extra_rs = rsketch_leg(torch.from_numpy(A_c2))
        del A_c2
        print("[bench] hashing / sampling done", file=sys.stderr, flush=True)
        if args.prec_rows > 0:
            extra_prec = precision_leg(args.prec_rows)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(d, l, n, seed, args.cpu_seconds)

    n_rr = int(sum(s_["n_reduce"] for s_ in st_bf))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": float(np.median(per)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f64",
        "data": "synthetic",
        "config": {"workload": "batch_512_random_noisy_fp32",
                   "sketches": S, "rows": total_rows, "d": "U{64..2048}", "l": "U{16..128}",
                   "n": "U{1000..50000}", "k": "l/2", "zeta": 10.0, "variant": "fd", "buffer_rows": "2l",
                   "products": "split-bf16 x3 Gram and rebuild, fp32 accumulation",
                   "eigensolver": "fp64 Householder tridiagonal + divide and conquer",
                   "launch": "per-class HIP graphs, replayed" if graph else
                             "direct launches, one stream per size class",
                   "reduce_steps": n_rr},
        "plain_fd_fp64_sequential": seq,
        "speedup_vs_plain_fd": value / seq["value"] if seq else None,
        "batch_fp64": {"value": total_rows / (ms64 / 1e3), "ms": ms64},
        ("batch_bf16x3_direct" if graph else "batch_bf16x3_graph"):
            {"value": total_rows / (ms_alt / 1e3), "ms_per_step": ms_alt,
             "ms_per_step_median": float(np.median(per_alt))},
        "roofline": roof,
        "tuning": tuning,
        "stages_batch_bf16x3": stages_bf,
        "stages_batch_fp64": stages_64,
        "profiled_step_ms": {"bf16x3": ms_p, "fp64": ms_p64},
        "parity": parity,
        "cpu_baseline": cpu,
        "single_stream": extra_single,
        "hashing_sampling": extra_rs,
        "precision_leg": extra_prec,
        "input_generation_s": t_gen,
    }
    print(json.dumps(out))
    if parity and any(isinstance(v, dict) and v.get("ok") is False for v in parity.values()):
        print("[bench] PARITY FAILED", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
