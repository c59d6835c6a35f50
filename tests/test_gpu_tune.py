"""Launch-shape tuning on the device: the tuner records a choice per size
bucket, every choice it can make gives the oracle's sketch (split-K counts
and slice lengths differ by rounding only; 32 and 64 rows per rebuild
workgroup give identical bits), and a batch's results stay independent of
how its sketches are grouped whatever slice length it was given."""
import numpy as np
import pytest

import oracle
from paper_1501_06561_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1501_06561_amd import fdsketch as F  # noqa: E402


@pytest.fixture
def tuner(tmp_path):
    old_path, old_mode = F.tune_path(), F.tune_mode()
    path = str(tmp_path / "tune.tsv")
    F.tune_path(path)
    F.tune_clear()
    yield path
    F.tune_clear()
    F.tune_path(old_path)
    F.tune_mode(old_mode)


def _dev():
    p = torch.cuda.get_device_properties(0)
    return f"{p.gcnArchName.split(':')[0]}/{p.multi_processor_count}"


def _pow2(x):
    b = 1
    while b < x:
        b *= 2
    return b


def _sizes(m, d):
    return f"|m{-(-m // 32) * 32}|d{_pow2(-(-d // 64) * 64)}"


def _single_keys(d, m, precision):
    g = {"fp64": 0, "bf16x3": 3, "fp8x3": 8}[precision]
    r = 0 if precision == "fp64" else 3
    s = _sizes(m, d)
    return f"{_dev()}|gram|p{g}{s}", f"{_dev()}|rebuild|p{r}{s}"


def _run_single(A, l, precision="fp64", buffer_rows=0, variant="fd"):
    sk = F.FDSketch(A.shape[1], l, variant, 0.2, precision=precision, buffer_rows=buffer_rows)
    sk.append(torch.from_numpy(A).cuda())
    B = sk.finalize().cpu().numpy()
    st = sk.stats()
    sk.close()
    return B, st


def test_refresh_records_a_choice_per_bucket_and_persists_it(tuner):
    F.tune_mode("refresh")
    A = synth.random_noisy(600, 1000, 20, 10.0, seed=(90, 0))
    _run_single(A, 100)
    kg, kr = _single_keys(1000, 200, "fp64")
    t = F.tune_table()
    assert kg in t and kr in t, t
    assert t[kg][0] in (1, 2, 4, 8) and t[kr][0] in (32, 64)
    assert all(":" in c for c in t[kg][1].split())          # candidate:microseconds notes
    F.tune_clear()
    F.tune_load(tuner)
    assert F.tune_table()[kg][0] == t[kg][0]


def test_off_mode_records_nothing(tuner):
    F.tune_mode("off")
    A = synth.random_noisy(300, 200, 10, 10.0, seed=(90, 1))
    _run_single(A, 40)
    assert F.tune_table() == {}


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_every_single_sketch_choice_matches_the_oracle(tuner, precision):
    """FD l = 100 on 3,000 x 1,000 rows with each split-K count the
    workspace holds and both rebuild tiles forced through the table."""
    F.tune_mode("on")
    A = synth.random_noisy(3000, 1000, 50, 10.0, seed=(91, 0))
    if precision != "fp64":
        A = synth.to_bf16(A).astype(np.float64)
    kg, kr = _single_keys(1000, 200, precision)
    Bo, so = oracle.fd_sketch(A, 100, "fd", return_state=True)
    fa = oracle.fro2(A)
    co = oracle.cov_err(A, Bo)
    results = {}
    for ks in (1, 2, 4, 8):
        for rt in (32, 64):
            F.tune_set(kg, ks)
            F.tune_set(kr, rt)
            B, st = _run_single(A, 100, precision)
            assert F.tune_lookup(kg) == ks and F.tune_lookup(kr) == rt
            assert st["n_reduce"] == so.n_rr
            ce = oracle.cov_err(A, B)
            if precision == "fp64":
                assert abs(ce - co) <= 1e-9 * co, (ks, rt, ce, co)
                assert np.max(np.abs(B.T @ B - Bo.T @ Bo)) <= 1e-9 * fa
            else:
                assert abs(ce - co) <= 1e-4, (ks, rt, ce, co)
            results[ks, rt] = B
    for ks in (1, 2, 4, 8):
        assert np.array_equal(results[ks, 32], results[ks, 64]), ks
    assert any(not np.array_equal(results[1, 32], results[k, 32]) for k in (2, 4, 8))


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_rebuild_tile_past_the_buffer_rows(tuner, precision):
    """buffer_rows = l + 1 = 71: 96 padded rows, 69 kept, so the last 64-row
    rebuild tile reaches past the padded rows (those rows of Ut read as
    zero)."""
    F.tune_mode("on")
    A = synth.random_noisy(1200, 300, 12, 10.0, seed=(92, 0))
    if precision != "fp64":
        A = synth.to_bf16(A).astype(np.float64)
    kg, kr = _single_keys(300, 71, precision)
    outs = []
    for rt in (32, 64):
        F.tune_set(kr, rt)
        B, st = _run_single(A, 70, precision, buffer_rows=71)
        outs.append(B)
    assert np.array_equal(outs[0], outs[1])
    Bo = oracle.fd_sketch(A, 70, "fd", m=71)
    ce, co = oracle.cov_err(A, outs[0]), oracle.cov_err(A, Bo)
    assert abs(ce - co) <= (1e-9 * co if precision == "fp64" else 1e-4), (ce, co)


def _size_class(m):
    return 0 if m <= 64 else (1 if m <= 128 else (2 if m <= 208 else 3))


def _batch_keys(cfgs):
    """bgram / brebuild keys of every (size class, precision) group."""
    groups = {}
    for c in cfgs:
        m = 2 * c["l"]
        q = 3 if c.get("precision", "fp64") == "bf16x3" else 0
        g = groups.setdefault((_size_class(m), q), [0, 0, 0])
        g[0] = max(g[0], -(-m // 32) * 32)
        g[1] = max(g[1], -(-c["d"] // 64) * 64)
        g[2] += 1
    keys = []
    for (_, q), (mp, ldc, n) in groups.items():
        s = f"|p{q}|m{mp}|d{_pow2(ldc)}|n{_pow2(n)}"
        keys.append((f"{_dev()}|bgram{s}", f"{_dev()}|brebuild{s}"))
    return keys


def _batch_cfgs(seed, S):
    rng = np.random.default_rng(seed)
    cfgs, mats = [], []
    for i in range(S):
        d = int(rng.integers(200, 2100))
        l = int(rng.integers(8, 129))
        n = int(rng.integers(100, 1200))
        A = synth.random_noisy(n, d, max(1, l // 2), 10.0, seed=(93, seed, i))
        p = "bf16x3" if i % 3 == 2 else "fp64"
        if p == "bf16x3":
            A = synth.to_bf16(A).astype(np.float64)
        cfgs.append(dict(d=d, l=l, variant="fd", alpha=0.2, precision=p))
        mats.append(A)
    return cfgs, mats


def _run_batch(cfgs, mats, grid=0):
    b = F.FDSketchBatch(cfgs)
    b.append([torch.from_numpy(A).cuda() for A in mats], grid_size=grid)
    outs = [o.cpu().numpy() for o in b.finalize(grid_size=grid)]
    stats = [b.stats(i) for i in range(len(cfgs))]
    b.close()
    return outs, stats


def test_every_batch_choice_matches_the_oracle_and_ignores_grouping(tuner):
    """Sketches of every size class, d up to 2,100 (up to eight K slices),
    FP64 and split-BF16 mixed; each slice length and rebuild tile forced
    through the table for every group."""
    F.tune_mode("on")
    cfgs, mats = _batch_cfgs(0, 18)
    keys = _batch_keys(cfgs)
    ref = [oracle.fd_sketch(A, c["l"], "fd", return_state=True) for c, A in zip(cfgs, mats)]
    by_kc = {}
    for kc in (0, 256, 512, 1024):
        per_rt = []
        for rt in (32, 64):
            for kg, kr in keys:
                F.tune_set(kg, kc)
                F.tune_set(kr, rt)
            outs, stats = _run_batch(cfgs, mats)
            for c, A, B, st, (Bo, so) in zip(cfgs, mats, outs, stats, ref):
                ce, co = oracle.cov_err(A, B), oracle.cov_err(A, Bo)
                tol = 1e-6 * co + 1e-12 if c["precision"] == "fp64" else 1e-4
                assert abs(ce - co) <= tol, (kc, rt, c, ce, co)
                assert st["n_reduce"] == so.n_rr
            per_rt.append(outs)
        for a, b in zip(*per_rt):
            assert np.array_equal(a, b), kc
        by_kc[kc] = per_rt[0]
        if kc == 256:
            one, _ = _run_batch(cfgs, mats, grid=1)
            for a, b in zip(per_rt[0], one):
                assert np.array_equal(a, b)
    # The slice length takes effect: some sketch's bits move with it.
    assert any(not np.array_equal(a, b) for a, b in zip(by_kc[0], by_kc[256]))


def test_batch_tuning_records_every_group(tuner):
    F.tune_mode("refresh")
    cfgs, mats = _batch_cfgs(1, 10)
    _run_batch(cfgs, mats)
    t = F.tune_table()
    for kg, kr in _batch_keys(cfgs):
        assert t[kg][0] in (0, 256, 512, 1024), (kg, t)
        if kr in t:
            assert t[kr][0] in (32, 64)
