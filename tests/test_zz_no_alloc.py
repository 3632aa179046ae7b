"""fst_cholesky_noalloc (scratch in the library's file-scope device array, no allocation)
against fst_cholesky (caller workspace) through the C ABI: two calls in a row, the second on
a smaller system, each equal to the workspace form (the same kernels, so bit for bit), and the
size limit rejected before any work."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
fst = pytest.importorskip("paper_1907_05884_amd.binding")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _spd(R, seed, dev):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((R + 40, R))
    return torch.from_numpy(A.T @ A + 1e-3 * np.eye(R)).to(dev)


def test_noalloc_cholesky_equals_workspace_form_twice(dev):
    lib = ctypes.CDLL(fst.LIB_PATH)
    assert hasattr(lib, "fst_cholesky_noalloc")
    for R, seed in ((1000, 1), (333, 2)):     # the second call is smaller than the first
        print(f"noalloc cholesky R={R} seed={seed}", flush=True)
        G = _spd(R, seed, dev)
        L_ref = G.clone()
        assert fst.fst_cholesky(L_ref) == 0
        L = G.clone()
        assert fst.fst_cholesky_noalloc(L) == 0
        torch.cuda.synchronize()
        low = torch.tril(torch.ones(R, R, dtype=torch.bool, device=dev))
        assert torch.equal(L[low], L_ref[low])
        # the stored diagonal-block inverses too: both solve identically
        b = torch.from_numpy(np.random.default_rng(seed + 10).standard_normal(R)).to(dev)
        x = fst.fst_cholesky_solve(L, b)
        x_ref = fst.fst_cholesky_solve(L_ref, b)
        assert torch.equal(x, x_ref)
        r = (G @ x - b).norm() / b.norm()
        assert r.item() <= 1e-10


def test_noalloc_cholesky_reports_breakdown_and_limit(dev):
    G = _spd(200, 3, dev)
    G[150, 150] = -1.0
    with pytest.raises(fst.FstError) as e:
        fst.fst_cholesky_noalloc(G)
    assert e.value.status == fst.FST_E_NOT_SPD
    # a later call after a breakdown starts from cleared flags
    H = _spd(300, 4, dev)
    H_ref = H.clone()
    fst.fst_cholesky(H_ref)
    assert fst.fst_cholesky_noalloc(H) == 0
    low = torch.tril(torch.ones(300, 300, dtype=torch.bool, device=dev))
    assert torch.equal(H[low], H_ref[low])
    # beyond the limit: rejected on the host before any launch (a 1-element tensor suffices)
    big = fst.FST_CHOLESKY_NOALLOC_MAX_R + 1
    st = fst._fn["fst_cholesky_noalloc"](big, fst._dev_ptr(torch.zeros(1, dtype=torch.float64, device=dev)),
                                         0.0, None, None)
    assert st == fst.FST_E_INVAL
    assert "outside" in fst.fst_last_error()
