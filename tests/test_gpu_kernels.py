"""Kernel-level parity: the device Gram product and Jacobi eigensolver against
NumPy/LAPACK on the same inputs (FP64)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1501_06561_amd import fdsketch as F  # noqa: E402


@pytest.mark.parametrize("rows,d", [(1, 5), (7, 3), (40, 100), (64, 64), (100, 1000), (130, 77),
                                    (512, 3072), (1024, 700)])
def test_gram_matches_numpy(rows, d):
    rng = np.random.default_rng(rows * 7 + d)
    C = rng.standard_normal((rows, d))
    G = F.gram(torch.from_numpy(C).cuda()).cpu().numpy()
    ref = C @ C.T
    assert np.max(np.abs(G - ref)) <= 1e-12 * np.max(np.abs(ref)) * max(1, d / 100)
    assert np.array_equal(G, G.T)


def _check_eigh(Gm, tol=1e-11, method="auto"):
    lam, V = F.eigh(torch.from_numpy(Gm).cuda(), method)
    lam, V = lam.cpu().numpy(), V.cpu().numpy()
    ref = np.linalg.eigvalsh(Gm)
    scale = max(np.max(np.abs(ref)), 1e-300)
    assert np.max(np.abs(np.sort(lam) - ref)) <= tol * scale
    m = Gm.shape[0]
    assert np.max(np.abs(V.T @ V - np.eye(m))) <= 1e-12 * m
    assert np.max(np.abs(Gm @ V - V * lam)) <= tol * scale
    return lam, V


# Orders at the edges of the register reduction's column groups (16 columns
# each, the last column k with k + 2 < m) and of its instances (64, 128, 192,
# 208 rows).
GROUP_EDGES = [4, 5, 17, 18, 19, 31, 32, 34, 48, 49, 50, 65, 66, 97, 113, 129, 145, 161, 177, 192, 193, 207]


@pytest.mark.parametrize("method", ["auto", "jacobi"])
@pytest.mark.parametrize("m", [1, 2, 3, 7, 33, 40, 64, 99, 100, 101, 128, 199, 200, 201, 208, 209, 230, 256, 257,
                               333, 400, 512, 513, 777, 1024] + GROUP_EDGES)
def test_eigh_random_psd(m, method):
    """"auto" is the tridiagonal divide-and-conquer route at every m (the
    matrix in registers up to 208; up to 256 the first m - 208 columns on the
    packed triangle in the workspace, the rest in registers; above 256 the
    full matrix in the workspace, two launches per column)."""
    if method == "jacobi" and m in [3, 33, 64, 199, 201, 208, 209, 230, 257, 400, 777] + GROUP_EDGES:
        pytest.skip("sizes added for the divide-and-conquer route")
    rng = np.random.default_rng(m)
    X = rng.standard_normal((m, 2 * m + 3)) * np.geomspace(1, 1e-3, 2 * m + 3)
    _check_eigh(X @ X.T, method=method)


@pytest.mark.parametrize("method", ["auto", "jacobi"])
@pytest.mark.parametrize("m", [17, 40, 130, 160, 200, 256, 400, 700])
def test_eigh_special_matrices(m, method):
    if method == "jacobi" and m in (17, 130, 400, 700):
        pytest.skip("size added for the divide-and-conquer route")
    rng = np.random.default_rng(m + 1)
    _check_eigh(np.diag(rng.uniform(0, 5, m)), method=method)       # already diagonal
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    lam = np.repeat([3.0, 1.0, 0.0], [m // 4, m // 4, m - 2 * (m // 4)])
    _check_eigh((Q * lam) @ Q.T, method=method)                       # repeated + zero
    _check_eigh(np.zeros((m, m)), method=method)
    X = rng.standard_normal((m, 5))
    _check_eigh(X @ X.T, method=method)                               # rank 5
    d = rng.uniform(1, 2, m)
    _check_eigh(np.diag(d) + 1e-9 * np.outer(d, d), method=method)    # clustered, near-diagonal
    _check_eigh(np.diag(np.r_[np.full(m // 2, 1e4), np.full(m - m // 2, 1e-6)]), method=method)  # two clusters


@pytest.mark.parametrize("precision,tol", [("bf16x3", 5e-5), ("bf16", 2e-2), ("fp8x3", 1e-2)])
@pytest.mark.parametrize("rows,d", [(40, 100), (130, 77), (512, 3072)])
def test_gram_reduced_precision(precision, tol, rows, d):
    """Reduced-precision matrix-core Gram: error bounded by the operand
    rounding times |c_i||c_j| -- one bf16 rounding ~2^-8 relative per
    element, split-bf16 ~2^-16; the per-row scaled e4m3 hi/lo split keeps
    each element to ~2^-8 of its row's largest magnitude."""
    rng = np.random.default_rng(rows + d)
    C = rng.standard_normal((rows, d)) * rng.uniform(0.5, 2.0, (rows, 1))
    G = F.gram(torch.from_numpy(C).cuda(), precision=precision).cpu().numpy()
    ref = C @ C.T
    nrm = np.sqrt(np.diag(ref))
    assert np.max(np.abs(G - ref) / np.outer(nrm, nrm)) <= tol
