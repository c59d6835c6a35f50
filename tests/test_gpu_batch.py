"""Many sketches advanced together in lock-step rounds: every sketch of a
batch against the oracle, and results independent of how the sketches are
grouped into launches or how the rows are split into append calls."""
import numpy as np
import pytest

import oracle
from paper_1501_06561_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1501_06561_amd import fdsketch as F  # noqa: E402

VARS = oracle.VARIANTS


def _make_batch(seed, S, d_range, l_range, n_range, variants=VARS, dtype=np.float64):
    rng = np.random.default_rng(seed)
    cfgs, mats = [], []
    for i in range(S):
        d = int(rng.integers(*d_range))
        l = int(rng.integers(*l_range))
        n = int(rng.integers(*n_range))
        v = variants[i % len(variants)]
        k = max(1, min(d - 1, l // 2))
        A = synth.random_noisy(n, d, k, 10.0, seed=(60, seed, i)).astype(dtype)
        cfgs.append(dict(d=d, l=l, variant=v, alpha=0.2))
        mats.append(A)
    return cfgs, mats


def _run(cfgs, mats, grid=0, chunks=1, dtype=torch.float64):
    b = F.FDSketchBatch(cfgs)
    tens = [torch.from_numpy(np.ascontiguousarray(A)).to(dtype).cuda() for A in mats]
    for c in range(chunks):
        parts = []
        for t in tens:
            n = t.shape[0]
            lo, hi = n * c // chunks, n * (c + 1) // chunks
            parts.append(t[lo:hi] if hi > lo else None)
        b.append(parts, grid_size=grid)
    outs = [o.cpu().numpy() for o in b.finalize(grid_size=grid)]
    stats = [b.stats(i) for i in range(len(cfgs))]
    b.close()
    return outs, stats


def _check(cfg, A, B, st, gram_tol):
    Bo, so = oracle.fd_sketch(A, cfg["l"], cfg["variant"], cfg["alpha"], return_state=True)
    fa = oracle.fro2(A)
    ce, co = oracle.cov_err(A, B), oracle.cov_err(A, Bo)
    assert abs(ce - co) <= 1e-6 * co + 1e-12, (cfg, ce, co)
    assert np.max(np.abs(B.T @ B - Bo.T @ Bo)) <= gram_tol * fa, cfg
    assert st["n_reduce"] == so.n_rr, cfg
    assert abs(st["fro2_A"] - so.fro2A) <= 1e-12 * fa
    assert abs(st["shrink_total"] - so.Stot) <= 1e-9 * fa
    assert st["eig_unconverged"] == 0


def test_batch_matches_oracle_mixed_shapes():
    """Buffer rows 8..256 (every size class of the tridiagonal reduction:
    registers only up to 208 rows, a packed-triangle head then registers
    above), d ragged against the 64-column padding, all four variants."""
    cfgs, mats = _make_batch(1, 24, (20, 300), (4, 129), (50, 2500))
    outs, stats = _run(cfgs, mats)
    for cfg, A, B, st in zip(cfgs, mats, outs, stats):
        _check(cfg, A, B, st, 1e-9 if cfg["variant"] == "fd" else 1e-7)


def test_batch_is_independent_of_grid_and_chunking():
    cfgs, mats = _make_batch(2, 12, (30, 200), (6, 90), (100, 1500))
    ref, _ = _run(cfgs, mats, grid=0)
    one, _ = _run(cfgs, mats, grid=1)
    chunked, _ = _run(cfgs, mats, grid=3, chunks=4)
    for a, b, c in zip(ref, one, chunked):
        assert np.array_equal(a, b)
        assert np.array_equal(a, c)


def test_batch_on_a_side_stream_waits_for_its_rows():
    """The batch created on a side stream, its rows produced on the current
    stream just before the append (a real dependency): the per-class streams
    start after the rows are ready, and the sketches equal those of a batch
    on the current stream, bit for bit.  Buffers in all four size classes."""
    cfgs = [dict(d=90, l=l, variant="fd", alpha=0.2) for l in (20, 50, 90, 120)]
    mats = [synth.random_noisy(900, 90, 5, 10.0, seed=(62, i)) for i in range(4)]
    ref, _ = _run(cfgs, mats)
    side = torch.cuda.Stream()
    b = F.FDSketchBatch(cfgs, stream=side)
    src = [torch.from_numpy(A).cuda() for A in mats]
    torch.cuda.synchronize()
    rows = [(t * 2.0) * 0.5 for t in src]          # made on the current stream
    b.append(rows)
    with torch.cuda.stream(side):
        outs = [o.cpu().numpy() for o in b.finalize()]
    b.close()
    for a, o in zip(ref, outs):
        assert np.array_equal(a, o)


def test_batch_edge_cases():
    cfgs = [dict(d=15, l=8, variant="fd", alpha=0.2),      # no rows
            dict(d=40, l=10, variant="alpha", alpha=0.2),  # fewer rows than l
            dict(d=33, l=1, variant="fd", alpha=0.2),      # l = 1
            dict(d=5, l=12, variant="isvd", alpha=0.2)]    # d < m
    mats = [np.zeros((0, 15)), synth.random_noisy(7, 40, 3, seed=(61, 1)),
            synth.random_noisy(300, 33, 3, seed=(61, 2)), synth.random_noisy(500, 5, 2, seed=(61, 3))]
    outs, stats = _run(cfgs, mats)
    assert not outs[0].any() and stats[0]["fro2_A"] == 0.0
    assert np.array_equal(outs[1][:7], mats[1]) and not outs[1][7:].any()
    assert not outs[2].any()
    for i in (1, 3):
        _check(cfgs[i], mats[i], outs[i], stats[i], 1e-8)


def test_batch_many_sketch_workload_draws():
    """First draws of the 512-sketch workload (d, l, n uniform), n capped so
    the oracle finishes; fp32 rows."""
    d, l, n = synth.batch_shapes(512, seed=(4, 0))
    cfgs, mats = [], []
    for i in range(16):
        nn = int(min(n[i], 1500))
        k = max(1, int(l[i]) // 2)
        A = synth.random_noisy(nn, int(d[i]), k, 10.0, seed=(4, 0, i)).astype(np.float32)
        cfgs.append(dict(d=int(d[i]), l=int(l[i]), variant="fd", alpha=0.2))
        mats.append(A)
    outs, stats = _run(cfgs, mats, dtype=torch.float32)
    for cfg, A, B, st in zip(cfgs, mats, outs, stats):
        _check(cfg, A.astype(np.float64), B, st, 1e-9)


def test_batch_rejects_large_buffers():
    with pytest.raises(F.FdskError) as e:
        F.FDSketchBatch([dict(d=10, l=129)])
    assert e.value.code == -6


def test_batch_reduced_precision_mixed():
    """Split-BF16 Gram and rebuild inside a batch that also holds FP64
    sketches: each sketch within its precision's bound of the FP64 oracle on
    the same bf16 rows (1e-4 for split-BF16, FP64's relative 1e-6)."""
    precs = ["fp64", "bf16x3", "fp64", "bf16x3"]
    cfgs, mats = [], []
    for i, p in enumerate(precs):
        A = synth.power_law(1500, 384, r=120, seed=(62, i), chunk=1500)
        mats.append(synth.to_bf16(A).astype(np.float64))
        cfgs.append(dict(d=384, l=24 + 8 * i, variant="fd", alpha=0.2, precision=p))
    b = F.FDSketchBatch(cfgs)
    b.append([torch.from_numpy(synth.bf16_bits(m.astype(np.float32)).view(np.int16)).view(torch.bfloat16).cuda()
              for m in mats])
    outs = [o.cpu().numpy() for o in b.finalize()]
    for i, (cfg, A, B) in enumerate(zip(cfgs, mats, outs)):
        Bo = oracle.fd_sketch(A, cfg["l"], "fd")
        ce, co = oracle.cov_err(A, B), oracle.cov_err(A, Bo)
        tol = {"fp64": 1e-6 * co + 1e-12, "bf16x3": 1e-4}[cfg["precision"]]
        assert abs(ce - co) <= tol, (cfg, ce, co)
        assert b.stats(i)["n_reduce"] == oracle.fd_sketch(A, cfg["l"], "fd", return_state=True)[1].n_rr
    b.close()


def test_batch_graph_capture_and_replay_match_direct_launches():
    """With graphs on, each append of a batch runs through HIP graphs captured
    per size class; after a reset an append with the same schedule replays
    them.  The sketches of
    the first (captured) call and of three replays, with eager GPU work and
    synchronisations in between, equal those of direct launches bit for bit.
    Buffers in all four size classes."""
    cfgs, mats = _make_batch(3, 12, (40, 260), (6, 128), (200, 1800))
    ref, ref_st = _run(cfgs, mats)
    b0 = F.FDSketchBatch(cfgs, graph=False)
    tens = [torch.from_numpy(A).cuda() for A in mats]
    b0.append(tens)
    direct = [o.cpu().numpy() for o in b0.finalize()]
    b0.close()
    b = F.FDSketchBatch(cfgs, graph=True)
    for rep in range(4):
        b.reset()
        b.append(tens)
        outs = [o.cpu().numpy() for o in b.finalize()]
        for i, (a, o) in enumerate(zip(direct, outs)):
            assert np.array_equal(a, o), (rep, i)
            st = b.stats(i)
            assert st["n_reduce"] == ref_st[i]["n_reduce"] and st["fro2_A"] == ref_st[i]["fro2_A"]
        torch.randn(1 << 20, device="cuda").sum().item()    # eager work between replays
    b.close()
    for a, o in zip(ref, direct):
        assert np.array_equal(a, o)


def test_batch_host_rows_match_device_rows():
    cfgs, mats = _make_batch(4, 6, (30, 150), (5, 60), (100, 900))
    ref, _ = _run(cfgs, mats)
    b = F.FDSketchBatch(cfgs)
    b.append([np.ascontiguousarray(A) for A in mats])
    outs = [o.cpu().numpy() for o in b.finalize()]
    b.close()
    for a, o in zip(ref, outs):
        assert np.array_equal(a, o)


def test_batch_profile_covers_every_stage():
    """FDSK_FLAG_PROFILE on a batch: every stage of the rounds is timed on the
    class streams with its algorithmic work, and the sketches are unchanged."""
    cfgs, mats = _make_batch(5, 8, (40, 300), (10, 128), (300, 1200), variants=("fd",))
    ref, _ = _run(cfgs, mats)
    b = F.FDSketchBatch(cfgs, profile=True)
    b.append([torch.from_numpy(A).cuda() for A in mats])
    outs = [o.cpu().numpy() for o in b.finalize()]
    prof = b.profile()
    b.close()
    for a, o in zip(ref, outs):
        assert np.array_equal(a, o)
    for stage in ("ingest", "gram", "eig", "tridiag", "dc", "backtr", "shrink", "rebuild"):
        ms, launches, work = prof[stage]
        assert launches > 0 and ms > 0, stage
        if stage != "shrink":
            assert work > 0, stage
    if any(2 * c["l"] > 208 for c in cfgs):    # buffers above 208 rows: the packed-triangle head
        assert prof["tridiag_head"][1] > 0


def test_batch_bf16x3_append_calls_match_one_call():
    """Split-BF16 sketches keep FP64 rows only where finalize may copy them
    out (rows no later ReduceRank of the same append call consumes).  Row
    counts per call chosen so that calls end right after a ReduceRank, on an
    exact buffer fill, in the middle of a fill, and so that finalize both
    reduces once more (more than l rows held) and copies the rows as they
    are (at most l held): every split gives the bits of one call."""
    shapes = [(96, 20), (130, 33), (64, 8), (200, 50)]
    cfgs, mats = [], []
    for i, (d, l) in enumerate(shapes):
        A = synth.to_bf16(synth.random_noisy(6 * l + 7 + i, d, max(1, l // 2), 10.0, seed=(64, i)))
        cfgs.append(dict(d=d, l=l, variant="fd", alpha=0.2, precision="bf16x3"))
        mats.append(A.astype(np.float64))
    ref = None
    for mode in ("one call", "chunks of l + 1", "exact fills"):
        b = F.FDSketchBatch(cfgs)
        tens = [torch.from_numpy(A).cuda() for A in mats]
        if mode == "one call":
            cuts = [[0, A.shape[0]] for A in mats]
        elif mode == "chunks of l + 1":
            cuts = [list(range(0, A.shape[0], l + 1)) + [A.shape[0]] for (d, l), A in zip(shapes, mats)]
        else:
            # 2l rows (an exact fill), then l + 1 (another exact fill), then the rest
            cuts = [[0, 2 * l, 3 * l + 1, A.shape[0]] for (d, l), A in zip(shapes, mats)]
        for c in range(max(len(x) for x in cuts) - 1):
            b.append([t[x[c]:x[c + 1]] if c + 1 < len(x) else None for t, x in zip(tens, cuts)])
        outs = [o.cpu().numpy() for o in b.finalize()]
        b.close()
        if ref is None:
            ref = outs
        else:
            for a, o in zip(ref, outs):
                assert np.array_equal(a, o), mode
    for cfg, A, B in zip(cfgs, mats, ref):
        Bo = oracle.fd_sketch(A, cfg["l"], "fd")
        ce, co = oracle.cov_err(A, B), oracle.cov_err(A, Bo)
        assert abs(ce - co) <= 1e-4, (cfg, ce, co)


def test_batch_bf16x3_finalize_without_a_last_reduction():
    """At most l rows held at finalize (no last ReduceRank): the FP64 rows
    copied out are the last ReduceRank's rows and the rows appended after
    it, split over several calls."""
    d, l = 120, 16
    A = synth.to_bf16(synth.random_noisy(2 * l + 1, d, 6, 10.0, seed=(65, 0))).astype(np.float64)
    cfg = [dict(d=d, l=l, variant="fd", alpha=0.2, precision="bf16x3")]
    # 2l rows: one ReduceRank, l - 1 rows kept; then 1 more row: l rows held.
    b = F.FDSketchBatch(cfg)
    t = torch.from_numpy(A).cuda()
    b.append([t[:2 * l]])
    b.append([t[2 * l:]])
    B = b.finalize()[0].cpu().numpy()
    st = b.stats(0)
    b.close()
    Bo, so = oracle.fd_sketch(A, l, "fd", return_state=True)
    assert st["n_reduce"] == so.n_rr == 1
    assert np.array_equal(B[l - 1], A[2 * l])     # the row appended after the reduction, as given
    ce, co = oracle.cov_err(A, B), oracle.cov_err(A, Bo)
    assert abs(ce - co) <= 1e-4, (ce, co)
