"""GPU parity of the hashing and sampling sketches (Hashing, OSNAP, Priority,
VarOpt; Sections 2.2 and 3.2) against the oracle on the same seeded rows and
the same counter-based random numbers.

Bars: Hashing and OSNAP sum the same terms as the oracle in another order
(FP64 atomics), so each entry of B is within 2 n eps of the sum of the
absolute values of its terms; the sampling sketches must keep exactly the
oracle's rows (indices compared as sets, and in order), with tau and the
rescaled rows within 1e-12 relative (the same arithmetic up to the order of
the row-norm sums)."""
import numpy as np
import pytest

import oracle
from oracle import rsketch as R
from paper_1501_06561_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1501_06561_amd import fdsketch as F  # noqa: E402

EPS = np.finfo(np.float64).eps


def _run(kind, A, l, s=4, key=0, chunks=None, dtype=torch.float64, host=False):
    """Append A in the given chunk sizes, then the rest (as oracle.rsketch)."""
    sk = F.RSketch(kind, A.shape[1], l, s=s, key=key)
    src = torch.from_numpy(np.ascontiguousarray(A)).to(dtype)
    if not host:
        src = src.cuda()
    n, lo, parts = A.shape[0], 0, []
    for c in chunks or []:
        parts.append((lo, min(lo + c, n)))
        lo = min(lo + c, n)
    parts.append((lo, n))
    for a, b in parts:
        if b > a:
            sk.append(src[a:b])
    B, idx = sk.finalize()
    st = sk.stats()
    sk.close()
    return B.cpu().numpy(), (None if idx is None else idx.cpu().numpy()), st


def _abs_sum_bound(A, l, s, key, kind):
    """Per entry of B: the sum of the absolute values of its terms."""
    inst = 1 if kind == "hash" else s
    rows = l // inst
    out = np.zeros((l, A.shape[1]))
    absA = np.abs(A)
    for i in range(A.shape[0]):
        for j in range(inst):
            out[j * rows + R.bucket(key, i, j, rows)] += absA[i] / np.sqrt(inst)
    return out


@pytest.mark.parametrize("kind,l,s", [("hash", 64, 1), ("hash", 7, 1), ("osnap", 64, 4), ("osnap", 30, 3)])
@pytest.mark.parametrize("chunks", [None, [1, 333, 1000]])
def test_hashing_matches_oracle(kind, l, s, chunks):
    A = synth.random_noisy(2500, 301, 8, 10.0, seed=(50, l))
    Bg, _, st = _run(kind, A, l, s, key=17, chunks=chunks)
    Bo, so = R.rsketch(A, kind, l, s=s, key=17, chunks=chunks)
    bound = 2 * A.shape[0] * EPS * _abs_sum_bound(A, l, s, 17, kind)
    assert np.all(np.abs(Bg - Bo) <= bound + 1e-300)
    assert abs(st["fro2_A"] - so.fro2A) <= 1e-12 * so.fro2A
    assert st["n_rows"] == 2500 and st["rows_kept"] == l


@pytest.mark.parametrize("kind", ["priority", "varopt"])
@pytest.mark.parametrize("l,chunks", [(40, None), (40, [1, 2, 3, 500, 999]), (1, [10, 10]), (333, [100, 900]),
                                      (3000, [1000])])
def test_sampling_matches_oracle(kind, l, chunks):
    """The kept rows (as indices, and in order), tau, the rescaled rows and
    the weight sum; l = 3,000 keeps every row of the 2,500."""
    A = synth.random_noisy(2500, 97, 6, 10.0, seed=(51, l)) * np.geomspace(0.05, 5.0, 2500)[:, None]
    Bg, ig, st = _run(kind, A, l, key=23, chunks=chunks)
    Bo, so = R.rsketch(A, kind, l, key=23, chunks=chunks)
    assert np.array_equal(ig, so.idx)
    assert abs(st["tau"] - so.tau) <= 1e-12 * max(so.tau, 1e-300)
    assert np.max(np.abs(Bg - Bo)) <= 1e-12 * np.max(np.abs(Bo))
    wsum = float(np.sum(so.adjusted_weights()))
    assert abs(st["weight_sum"] - wsum) <= 1e-12 * wsum
    if kind == "varopt":
        assert abs(st["weight_sum"] - st["fro2_A"]) <= 1e-12 * st["fro2_A"]


@pytest.mark.parametrize("kind", ["hash", "osnap", "priority", "varopt"])
def test_input_dtypes_and_host_rows(kind):
    A = synth.random_noisy(800, 64, 4, 10.0, seed=(52, 0)).astype(np.float32).astype(np.float64)
    ref, iref, _ = _run(kind, A, 32, key=5, chunks=[300])
    for dtype, host in ((torch.float32, False), (torch.float64, True)):
        B, idx, _ = _run(kind, A, 32, key=5, chunks=[300], dtype=dtype, host=host)
        if kind in ("hash", "osnap"):
            assert np.allclose(B, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        else:
            assert np.array_equal(idx, iref)
            assert np.allclose(B, ref, rtol=1e-13, atol=0)


def test_covariance_error_of_each_sketch_against_the_oracle_evaluator():
    """cov-err of each GPU sketch (the oracle's dense evaluator) equals that
    of the oracle's sketch."""
    A = synth.random_noisy(4000, 120, 10, 10.0, seed=(53, 0))
    for kind in ("hash", "osnap", "priority", "varopt"):
        Bg, _, _ = _run(kind, A, 200, key=31, chunks=[1500])
        Bo, _ = R.rsketch(A, kind, 200, key=31, chunks=[1500])
        cg, co = oracle.cov_err(A, Bg), oracle.cov_err(A, Bo)
        assert abs(cg - co) <= 1e-9 * co, (kind, cg, co)
