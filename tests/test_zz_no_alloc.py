"""fdsk_eigh_noalloc (the eigensolve on the library's static device scratch,
no allocation) against fdsk_eigh on the same inputs, through the C ABI: two
calls in a row, the second on a smaller matrix (so it runs on scratch the
first one left behind), then the largest size the scratch takes."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1501_06561_amd import fdsketch as F  # noqa: E402


def _sym(m, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, 2 * m + 5)) * np.geomspace(1, 1e-3, 2 * m + 5)
    return X @ X.T


def _eigh_c(fn, Gm, noalloc):
    m = Gm.shape[0]
    G = torch.from_numpy(Gm).cuda()
    lam = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
    V = torch.full((m, m), np.nan, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [ctypes.c_void_p(G.data_ptr()), m, G.stride(0), ctypes.c_void_p(lam.data_ptr()),
            ctypes.c_void_p(V.data_ptr()), V.stride(0)]
    rc = fn(*args, stream) if noalloc else fn(*args, 0, stream)
    assert rc == 0, F.lib().sketch_last_error(None)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), V.cpu().numpy()


@pytest.mark.parametrize("sizes", [(300, 120), (200, 64)])
def test_noalloc_eigh_matches_allocating_entry_point(sizes):
    L = F.lib()
    for i, m in enumerate(sizes + (512,)):
        Gm = _sym(m, 100 * i + m)
        lam_a, V_a = _eigh_c(L.fdsk_eigh, Gm, noalloc=False)
        lam_n, V_n = _eigh_c(L.fdsk_eigh_noalloc, Gm, noalloc=True)
        assert np.array_equal(lam_a, lam_n), m
        assert np.array_equal(V_a, V_n), m
        scale = np.max(np.abs(lam_a))
        assert np.max(np.abs(Gm @ V_n - V_n * lam_n)) <= 1e-11 * scale


def test_noalloc_eigh_rejects_sizes_beyond_its_scratch():
    L = F.lib()
    G = torch.zeros((513, 513), dtype=torch.float64, device="cuda")
    lam = torch.zeros(513, dtype=torch.float64, device="cuda")
    rc = L.fdsk_eigh_noalloc(ctypes.c_void_p(G.data_ptr()), 513, 513, ctypes.c_void_p(lam.data_ptr()),
                             ctypes.c_void_p(G.data_ptr()), 513, None)
    assert rc == -6
    assert b"scratch" in L.sketch_last_error(None)
