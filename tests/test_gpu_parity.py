"""GPU parity of every hot-path step against the FP64 oracle, through the C ABI.

Tolerances (relative L2 over the compared vector): FP64 paths 1e-10; FP32 paths 1e-5 for
factor values, Gram entries and reconstructed values.  The FP32 core is compared with a
bound that scales with the conditioning of the sampled Gram (perturbation bound
||d alpha|| / ||alpha|| <= kappa(G) ||dG|| / ||G||, with ||dG|| / ||G|| ~ 1e-7 for FP32 rows).
FP32 inputs are compared against the oracle evaluated at the same float32 numbers up-cast
exactly to float64, so the comparison measures kernel arithmetic only.
"""
import numpy as np
import pytest

import datagen
from oracle import lsq, pipeline, reconstruct
from oracle.model import Model as OModel
from oracle.reconstruct import rel_l2
from oracle.sampler import STREAM_LS, sample_without_replacement

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
fst = pytest.importorskip("paper_1907_05884_amd.binding")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def D(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def H(t):
    return t.detach().cpu().numpy()


def _pts(seed, n, lo=(-1, -1, -1), hi=(1, 1, 1), dtype=np.float64):
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return (lo + (hi - lo) * rng.random((n, 3))).astype(dtype)


def _models(seed, rank, degree, lo=(-1, -1, -1), hi=(1, 1, 1)):
    core, coefs = datagen.random_model_parts(seed, rank, degree)
    om = OModel(tuple(lo), tuple(hi), tuple(rank), tuple(degree), core, coefs)
    gm = fst.fst_model_from_parts(lo, hi, rank, degree, core, coefs)
    return om, gm


def _soa(p, dev):
    return [D(np.ascontiguousarray(p[:, k]), dev) for k in range(3)]


# ------------------------------------------------------------------------------ factor values
@pytest.mark.parametrize("dtype,rank,degree,n,m,tol", [
    (np.float64, (5, 7, 3), (9, 12, 6), 3001, 1337, 1e-10),
    (np.float64, (8, 8, 8), (15, 15, 15), 20000, 2000, 1e-10),
    (np.float32, (24, 24, 24), (31, 31, 31), 50001, 20011, 1e-5),
    (np.float32, (32, 4, 17), (31, 15, 20), 9000, 9000, 1e-5),
    (np.float32, (16, 12, 9), (15, 9, 12), 7001, 5003, 1e-5),      # 16 basis values, one column block
    (np.float32, (5, 7, 3), (9, 12, 6), 4097, 4097, 1e-5),
])
def test_factor_eval_parity(dev, dtype, rank, degree, n, m, tol):
    om, gm = _models(1, rank, degree, lo=(0, 0, 0), hi=(4, 1, 1))
    pts = _pts(2, n, (0, 0, 0), (4, 1, 1), dtype)
    v = np.random.default_rng(3).standard_normal(n).astype(dtype)
    idx = np.sort(np.random.default_rng(4).choice(n, m, replace=False)).astype(np.int32)
    x, y, z = _soa(pts, dev)
    U, vs = fst.fst_factor_eval(gm, x, y, z, D(v, dev), D(idx, dev))
    ref = lsq.factor_values(om, pts[idx].astype(np.float64))
    Uh = H(U)
    off = 0
    for k in range(3):
        assert rel_l2(Uh[off:off + rank[k]].T, ref[k]) <= tol
        off += rank[k]
    np.testing.assert_array_equal(H(vs), v[idx])


# ------------------------------------------------------------------------------ Gram and A^T v
def _gram_case(dev, dtype, rank, degree, m, seed=5):
    om, gm = _models(seed, rank, degree)
    pts = _pts(seed + 1, m, dtype=dtype)
    v = np.random.default_rng(seed + 2).standard_normal(m).astype(dtype)
    x, y, z = _soa(pts, dev)
    U, vs = fst.fst_factor_eval(gm, x, y, z, D(v, dev))
    G, h = fst.fst_gram(gm, U, vs)
    Gr, hr = lsq.normal_equations(om, pts.astype(np.float64), v.astype(np.float64))
    return H(G), H(h), Gr, hr


@pytest.mark.parametrize("rank,degree,m", [((5, 7, 3), (9, 12, 6), 777), ((8, 8, 8), (15, 15, 15), 2037),
                                           ((9, 10, 11), (13, 9, 11), 3001), ((1, 1, 1), (0, 3, 2), 50)])
def test_gram_fp64_parity(dev, rank, degree, m):
    G, h, Gr, hr = _gram_case(dev, np.float64, rank, degree, m)
    low = np.tril_indices(Gr.shape[0])
    assert rel_l2(G[low], Gr[low]) <= 1e-10
    assert rel_l2(h, hr) <= 1e-10


@pytest.mark.parametrize("rank,degree,m", [((12, 11, 10), (20, 20, 20), 20013), ((6, 6, 6), (31, 31, 31), 4099)])
def test_gram_fp32_parity(dev, rank, degree, m):
    G, h, Gr, hr = _gram_case(dev, np.float32, rank, degree, m)
    low = np.tril_indices(Gr.shape[0])
    assert rel_l2(G[low], Gr[low]) <= 1e-5
    assert rel_l2(h, hr) <= 1e-5


def test_gram_kronecker_closed_form(dev):
    from oracle.interp import grid_nodes, grid_points
    from oracle.basis import legendre_orthonormal
    rank, degree, grid = (3, 4, 2), (6, 5, 7), (5, 6, 7)
    om, gm = _models(8, rank, degree)
    pts = grid_points(grid)
    x, y, z = _soa(pts, dev)
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    G, _ = fst.fst_gram(gm, U)
    Uk = [legendre_orthonormal(grid_nodes(I), degree[k]) @ om.coefs[k] for k, I in enumerate(grid)]
    K = np.kron(np.kron(Uk[0].T @ Uk[0], Uk[1].T @ Uk[1]), Uk[2].T @ Uk[2])
    low = np.tril_indices(K.shape[0])
    assert rel_l2(H(G)[low], K[low]) <= 1e-12


def test_gram_is_deterministic(dev):
    om, gm = _models(9, (10, 9, 8), (15, 15, 15))
    pts = _pts(10, 30000, dtype=np.float32)
    x, y, z = _soa(pts, dev)
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    G1, _ = fst.fst_gram(gm, U)
    G2, _ = fst.fst_gram(gm, U)
    assert torch.equal(G1, G2)


# dense route of fst_gram: design rows materialised transposed in the workspace, then the
# dense MFMA Gram; one chunk holding every row, or 4096-row chunks with a ragged last one
@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-10), (np.float32, 1e-5)])
@pytest.mark.parametrize("rank,degree,m", [((5, 7, 3), (9, 12, 6), 777), ((12, 11, 10), (20, 20, 20), 9001),
                                           ((12, 11, 10), (20, 20, 20), 9004)])
@pytest.mark.parametrize("chunked", [False, True])
def test_gram_dense_route_parity(dev, dtype, tol, rank, degree, m, chunked):
    om, gm = _models(31, rank, degree)
    pts = _pts(32, m, dtype=dtype)
    x, y, z = _soa(pts, dev)
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    code = fst.FST_F64 if dtype == np.float64 else fst.FST_F32
    base = fst.fst_gram_workspace_bytes(gm, m)
    full = fst.fst_gram_dense_workspace_bytes(gm, code, m)
    assert full > base
    size = base + np.dtype(dtype).itemsize * gm.R * 4096 + 100 if chunked else full
    ws = torch.empty(size, dtype=torch.uint8, device=dev)
    G, _ = fst.fst_gram(gm, U, ws=ws)
    Gk, _ = fst.fst_gram(gm, U)                   # the Khatri-Rao route (minimal workspace)
    Gr, _ = lsq.normal_equations(om, pts.astype(np.float64), np.zeros(m))
    low = np.tril_indices(Gr.shape[0])
    assert rel_l2(H(G)[low], Gr[low]) <= tol
    assert rel_l2(H(G)[low], H(Gk)[low]) <= tol
    G2, _ = fst.fst_gram(gm, U, ws=ws)
    assert torch.equal(G, G2)


# dense route of the 16-bit Gram: the same 16-bit entries ((u1 u2) scale) u3 and the same
# 16x16x32 MFMA sums per 128-point chunk as the Khatri-Rao precision-form kernel, so the two
# Grams are equal bit for bit (row counts with and without 16-byte loads, r3 < 8)
@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("rank,degree,m", [((12, 11, 10), (20, 20, 20), 9004), ((5, 7, 3), (9, 12, 6), 777),
                                           ((9, 8, 5), (15, 15, 15), 4101)])
def test_gram_16bit_dense_route_equals_khatri_rao(dev, prec, rank, degree, m):
    code = {"bf16": fst.FST_GRAM_BF16, "f16": fst.FST_GRAM_F16}[prec]
    om, gm = _models(33, rank, degree)
    pts = _pts(34, m, dtype=np.float32)
    x, y, z = _soa(pts, dev)
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    Gk, _ = fst.fst_gram(gm, U, gram_prec=code)
    ws = torch.empty(fst.fst_gram_dense_workspace_bytes(gm, fst.FST_F32, m), dtype=torch.uint8, device=dev)
    Gd, _ = fst.fst_gram(gm, U, gram_prec=code, ws=ws)
    low = torch.tril(torch.ones_like(Gk, dtype=torch.bool))
    assert torch.equal(Gd[low], Gk[low])


def test_refit_dense_route_matches_oracle(dev):
    w, m0 = _small_workload_model()
    alpha_o, _, _, _ = lsq.refit_core(m0, w.pts, w.vals, w.n_samples, w.seed)
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, m0.core, m0.coefs)
    x, y, z, v = [D(a, dev) for a in w.soa()]
    extra = fst.fst_gram_dense_workspace_bytes(gm, fst.FST_F64, w.n_samples)
    ws = torch.empty(fst.fst_refit_workspace_bytes(gm, fst.FST_F64, w.n_samples) + extra, dtype=torch.uint8,
                     device=dev)
    out = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed, ws=ws)
    assert rel_l2(out.core, alpha_o) <= 1e-10


# ------------------------------------------------------------------------------ Cholesky + solve
# sizes cover one block, a ragged last block, trailing updates whose last row block is
# shorter than a tile (R - base not a multiple of 256) and several 256-column panels
@pytest.mark.parametrize("R", [1, 64, 65, 257, 300, 333, 1000, 4097])
def test_cholesky_and_solve(dev, R):
    rng = np.random.default_rng(R)
    B = rng.standard_normal((R, R))
    A = B @ B.T / R + np.eye(R)
    b = rng.standard_normal(R)
    G = D(A.copy(), dev)
    assert fst.fst_cholesky(G) == 0
    Gh = H(G)
    Lref = np.linalg.cholesky(A)
    assert rel_l2(np.tril(Gh), Lref) <= 1e-12
    # strict upper triangle of every 64 x 64 diagonal block: its inverse, transposed
    for k0 in range(0, R, 64):
        nb = min(64, R - k0)
        inv = np.linalg.inv(Lref[k0:k0 + nb, k0:k0 + nb])
        got = np.triu(Gh[k0:k0 + nb, k0:k0 + nb], 1).T
        assert np.abs(got - np.tril(inv, -1)).max() <= 1e-12 * np.abs(inv).max()
    x = fst.fst_cholesky_solve(G, D(b, dev))
    assert rel_l2(H(x), np.linalg.solve(A, b)) <= 1e-10


def test_cholesky_with_diagonal_shift(dev):
    # G + s diag(G) = L L^T
    R = 300
    rng = np.random.default_rng(5)
    B = rng.standard_normal((R, R))
    A = B @ B.T / R + 0.1 * np.eye(R)
    s = 1e-3
    G = D(A.copy(), dev)
    assert fst.fst_cholesky(G, shift=s) == 0
    As = A + s * np.diag(np.diag(A))
    assert rel_l2(np.tril(H(G)), np.linalg.cholesky(As)) <= 1e-12
    with pytest.raises(fst.FstError):
        fst.fst_cholesky(D(A.copy(), dev), shift=-1.0)


def test_cholesky_reports_non_spd_pivot(dev):
    R = 200
    A = np.eye(R)
    A[137, 137] = -1.0
    with pytest.raises(fst.FstError) as e:
        fst.fst_cholesky(D(A, dev))
    assert e.value.status == fst.FST_E_NOT_SPD
    assert "info=138" in str(e.value)


# ------------------------------------------------------------------------------ reconstruction
@pytest.mark.parametrize("dtype,rank,degree,n,tol", [
    (np.float64, (8, 8, 8), (15, 15, 15), 20001, 1e-10),
    (np.float64, (5, 7, 3), (9, 12, 6), 4097, 1e-10),
    (np.float64, (24, 24, 24), (31, 31, 31), 3000, 1e-10),
    (np.float32, (24, 24, 24), (31, 31, 31), 100003, 1e-5),
    (np.float32, (32, 32, 32), (31, 31, 31), 5000, 1e-5),
    (np.float32, (4, 20, 9), (15, 31, 22), 777, 1e-5),
    (np.float32, (7, 5, 11), (12, 9, 20), 4999, 1e-5),     # r2 < 16, r3 not a multiple of 4
    (np.float32, (30, 3, 2), (31, 4, 2), 2500, 1e-5),      # r1 r2 = 90: a partial 16-column block
    (np.float32, (1, 1, 1), (0, 0, 0), 1, 1e-6),
    # instances of the MFMA kernel by padded rank and degree steps per column block
    (np.float32, (16, 16, 16), (31, 31, 31), 30001, 1e-5),   # ranks padded to 16, 2 steps per block
    (np.float32, (12, 20, 17), (25, 31, 19), 20011, 1e-5),   # ranks padded to 24, 2 steps per block
    (np.float32, (8, 8, 8), (15, 15, 15), 20001, 1e-5),      # ranks padded to 8, 4 steps per block
    (np.float32, (32, 16, 8), (31, 20, 11), 9001, 1e-5),     # ranks padded to 32, 1 step per block
])
def test_eval_parity(dev, dtype, rank, degree, n, tol):
    om, gm = _models(11, rank, degree, lo=(0, 0, 0), hi=(4, 1, 1))
    pts = _pts(12, n, (0, 0, 0), (4, 1, 1), dtype)
    x, y, z = _soa(pts, dev)
    f = fst.fst_eval(gm, x, y, z)
    ref = reconstruct.evaluate(om, pts.astype(np.float64))
    assert rel_l2(H(f), ref) <= tol


def test_eval_empty(dev):
    _, gm = _models(1, (2, 2, 2), (3, 3, 3))
    e = torch.empty(0, dtype=torch.float32, device=dev)
    assert fst.fst_eval(gm, e, e, e).numel() == 0


@pytest.mark.parametrize("dtype,n,tol", [(np.float64, 20001, 1e-10), (np.float32, 300007, 1e-5)])
def test_eval_error_parity(dev, dtype, n, tol):
    # sums of (v - f)^2 and v^2 against the oracle's reconstruction of the same points; the
    # values are the field plus noise, so the data error is neither 0 nor 1
    om, gm = _models(17, (7, 6, 5), (12, 12, 12))
    pts = _pts(18, n, dtype=dtype)
    p64 = pts.astype(np.float64)
    f = reconstruct.evaluate(om, p64)
    v = (f + 0.05 * np.std(f) * np.random.default_rng(19).standard_normal(n)).astype(dtype)
    x, y, z = _soa(pts, dev)
    s_err, s_v = fst.fst_eval_error(gm, x, y, z, D(v, dev))
    v64 = v.astype(np.float64)
    ref_err, ref_v = float(np.sum((v64 - f) ** 2)), float(np.sum(v64 ** 2))
    assert abs(s_v - ref_v) <= 1e-12 * ref_v
    # FP32 reconstruction errors (~1e-7 of |f|) against a residual of 5%: rel 1e-5 on the sum
    assert abs(s_err - ref_err) <= tol * ref_err
    assert np.sqrt(s_err / s_v) == pytest.approx(np.linalg.norm(v64 - f) / np.linalg.norm(v64), rel=tol)
    # deterministic: the same bits twice
    assert fst.fst_eval_error(gm, x, y, z, D(v, dev)) == (s_err, s_v)


# ------------------------------------------------------------------------------ FP64 residual
def test_residual_fp64_parity(dev):
    om, gm = _models(13, (6, 5, 4), (10, 10, 10))
    n, m = 5000, 1200
    pts = _pts(14, n, dtype=np.float32)
    v = np.random.default_rng(15).standard_normal(n).astype(np.float32)
    idx = np.sort(np.random.default_rng(16).choice(n, m, replace=False)).astype(np.int32)
    alpha = np.random.default_rng(17).standard_normal(om.R)
    x, y, z = _soa(pts, dev)
    r = fst.fst_residual(gm, x, y, z, D(v, dev), D(idx, dev), D(alpha, dev))
    ref = lsq.residual_normal(om, pts[idx].astype(np.float64), v[idx].astype(np.float64), alpha)
    assert rel_l2(H(r), ref) <= 1e-10


# ------------------------------------------------------------------------------ Algorithm 2 end to end
def _small_workload_model():
    w = datagen.small_f64()
    m0 = pipeline.compress(w.pts, w.vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction, w.seed)
    return w, m0


def test_refit_core_fp64_matches_oracle(dev):
    w, m0 = _small_workload_model()
    alpha_o, idx, G, h = lsq.refit_core(m0, w.pts, w.vals, w.n_samples, w.seed)
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, m0.core, m0.coefs)
    x, y, z, v = [D(a, dev) for a in w.soa()]
    out = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed)
    assert rel_l2(out.core, alpha_o) <= 1e-10
    f = fst.fst_eval(out, x, y, z)
    ref = reconstruct.evaluate(m0.with_core(alpha_o), w.pts)
    assert rel_l2(H(f), ref) <= 1e-10


def test_fit_end_to_end_fp64(dev):
    w = datagen.small_f64()
    mo = pipeline.fit(w.pts, w.vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction,
                      w.n_samples, w.seed)
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=w.grid, rank=w.rank, degree=w.degree,
                        interp_fraction=w.interp_fraction, n_samples=w.n_samples, seed=w.seed)
    x, y, z, v = [D(a, dev) for a in w.soa()]
    gm = fst.fst_fit(p, x, y, z, v)
    for k in range(3):
        np.testing.assert_array_equal(gm.coefs(k) != 0, mo.coefs[k] != 0)
        assert rel_l2(gm.coefs(k), mo.coefs[k]) <= 1e-10
    print(f"core rel-L2 {rel_l2(gm.core, mo.core):.3e}", flush=True)
    assert rel_l2(gm.core, mo.core) <= 1e-10
    f = H(fst.fst_eval(gm, x, y, z))
    err_gpu, err_ref = rel_l2(f, w.vals), rel_l2(reconstruct.evaluate(mo, w.pts), w.vals)
    assert abs(err_gpu - err_ref) <= 1e-8 * err_ref + 1e-12


def test_fit_end_to_end_lars_fp64(dev):
    # Algorithm 1 with the paper's sparse solver (Lasso-LARS + leave-one-out), then Algorithm 2
    w = datagen.small_f64()
    mo = pipeline.fit(w.pts, w.vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction,
                      w.n_samples, w.seed, solver="lars")
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=w.grid, rank=w.rank, degree=w.degree,
                        interp_fraction=w.interp_fraction, n_samples=w.n_samples, seed=w.seed,
                        sparse_solver=fst.FST_SOLVER_LARS)
    x, y, z, v = [D(a, dev) for a in w.soa()]
    gm = fst.fst_fit(p, x, y, z, v)
    for k in range(3):
        np.testing.assert_array_equal(gm.coefs(k) != 0, mo.coefs[k] != 0)
        assert rel_l2(gm.coefs(k), mo.coefs[k]) <= 1e-10
    print(f"core rel-L2 {rel_l2(gm.core, mo.core):.3e}", flush=True)
    assert rel_l2(gm.core, mo.core) <= 1e-10


def test_fit_with_ranks_from_precision(dev):
    # Algorithm 1 with ranks chosen from eps (Sec. 4.1, Table 1), then Algorithm 2: the ranks
    # the oracle's rule picks on its interpolated grid, and the oracle's fit at those ranks
    from oracle.sthosvd import ranks_for_precision
    w = datagen.small_f64()
    eps, caps = 0.1, (10, 10, 10)
    T = pipeline.compress(w.pts, w.vals, w.lo, w.hi, w.grid, (1, 1, 1), w.degree, w.interp_fraction,
                          w.seed).info["grid_tensor"]
    r = tuple(min(a, c) for a, c in zip(ranks_for_precision(T, eps), caps))
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=w.grid, rank=caps, degree=w.degree,
                        interp_fraction=w.interp_fraction, n_samples=w.n_samples, seed=w.seed, eps=eps)
    x, y, z, v = [D(a, dev) for a in w.soa()]
    gm = fst.fst_fit(p, x, y, z, v)
    assert gm.info()["rank"] == r
    mo = pipeline.fit(w.pts, w.vals, w.lo, w.hi, w.grid, r, w.degree, w.interp_fraction, w.n_samples, w.seed)
    print(f"core rel-L2 {rel_l2(gm.core, mo.core):.3e}", flush=True)
    assert rel_l2(gm.core, mo.core) <= 1e-10


def test_refit_rejects_too_few_samples_and_solves_rank_one_design(dev):
    om, gm = _models(20, (4, 4, 4), (6, 6, 6))
    pts = _pts(21, 500)
    x, y, z = _soa(pts, dev)
    v = D(np.full(500, 1.5), dev)
    with pytest.raises(fst.FstError) as e:
        fst.fst_refit_core(gm, x, y, z, v, 64, 1)
    assert e.value.status == fst.FST_E_INVAL
    # every point identical: the sampled design has rank one.  The strict Cholesky breaks
    # down, the FP64 step keeps the first column and drops the other R - 1 as dependent,
    # and the field at the point equals the value
    same = [D(np.full(500, 0.3), dev) for _ in range(3)]
    out = fst.fst_refit_core(gm, *same, v, 200, 1)
    prec, dropped = out.fit_info()
    assert prec == fst.FST_GRAM_F64 and dropped == om.R - 1
    assert np.count_nonzero(out.core) == 1
    f = H(fst.fst_eval(out, *[t[:1].contiguous() for t in same]))
    assert abs(f[0] - 1.5) <= 1e-12


def test_refit_exact_recovery_fp32(dev):
    # a field that lies in the model span: the sampled LS must return the planted core
    om, gm = _models(22, (10, 9, 8), (15, 15, 15))
    n, M = 60000, 6000
    pts = _pts(23, n, dtype=np.float32)
    idx = sample_without_replacement(7, STREAM_LS, n, M)
    v = np.zeros(n, dtype=np.float64)
    v[idx] = reconstruct.evaluate(om, pts[idx].astype(np.float64))
    x, y, z = _soa(pts, dev)
    out = fst.fst_refit_core(gm, x, y, z, D(v.astype(np.float32), dev), M, 7)
    G, _ = lsq.normal_equations(om, pts[idx].astype(np.float64), v[idx])
    kappa = np.linalg.cond(G)
    assert rel_l2(out.core, om.core) <= max(1e-5, 1e-6 * kappa)


# ------------------------------------------------------------------------------ precision form
@pytest.mark.parametrize("rank", [(9, 8, 7), (12, 10, 9)])
@pytest.mark.parametrize("prec,u", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)])
def test_gram_16bit_within_rounding_bound(dev, prec, u, rank):
    # each design-row entry is rounded once to the 16-bit format, so every Gram entry is within
    # ~2u * sum_q |A[q,j] A[q,j']| of the exact value (plus FP32 accumulation, far smaller).
    # r3 = 7 forms entries from three factors, r3 = 9 from (j1, j2) pair tables; R = 1080
    # spans five 256-wide tiles with a ragged edge.
    code = fst.FST_GRAM_BF16 if prec == "bf16" else fst.FST_GRAM_F16
    om, gm = _models(30, rank, (15, 15, 15))
    m = 6007
    pts = _pts(31, m, dtype=np.float32)
    x, y, z = _soa(pts, dev)
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    G, _ = fst.fst_gram(gm, U, gram_prec=code)
    A = lsq.design_rows(lsq.factor_values(om, pts.astype(np.float64)))
    Gr = A.T @ A
    bound = np.abs(A).T @ np.abs(A)
    low = np.tril_indices(om.R)
    err = np.abs(H(G)[low] - Gr[low])
    assert np.all(err <= 2.2 * u * bound[low] + 1e-12 * np.abs(Gr).max())
    assert rel_l2(H(G)[low], Gr[low]) <= 4 * u


@pytest.mark.parametrize("prec", [fst.FST_GRAM_BF16, fst.FST_GRAM_F16])
def test_refit_16bit_gram_with_refinement_matches_fp64(dev, prec):
    w, m0 = _small_workload_model()
    n = 40000
    wl = datagen.make_workload("lp", seed=3, n=n, n_gauss=6, grid=(32, 32, 32), rank=(8, 8, 8),
                               degree=(15, 15, 15), interp_fraction=0.1, n_samples=4000, dtype=np.float32)
    alpha_o, idx, G, h = lsq.refit_core(m0, wl.pts.astype(np.float64), wl.vals.astype(np.float64), 4000, 9)
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, m0.core, m0.coefs)
    x, y, z, v = [D(a, dev) for a in wl.soa()]
    errs, res = [], []
    for steps in (0, 1, 3):
        out = fst.fst_refit_core(gm, x, y, z, v, 4000, 9, gram_prec=prec, refine_steps=steps)
        errs.append(rel_l2(out.core, alpha_o))
        info = out.solve_info()
        assert info["dropped"] == 0 and info["refine_steps"] <= 4 * steps
        res.append(info["rel_residual"])
        # a refinement that ends above a relative residual of 1e-8 (after the steps asked for,
        # and further steps while each halves the residual, at most 4 x steps) climbs the
        # precision ladder to FP32 rows; otherwise the core keeps the 16-bit Gram
        if steps == 0:
            assert info["gram_prec"] == prec
        else:
            assert (info["gram_prec"] == prec and info["rel_residual"] <= 1e-8) or \
                info["gram_prec"] == fst.FST_GRAM_F32, info
    assert errs[2] <= 1e-6, errs
    assert errs[2] < errs[0], errs
    assert np.isnan(res[0]) and res[2] <= 1e-8, res
    # many steps: refinement stops once a step no longer reduces the FP64 residual
    out = fst.fst_refit_core(gm, x, y, z, v, 4000, 9, gram_prec=prec, refine_steps=40)
    info = out.solve_info()
    assert info["refine_steps"] < 40 and info["rel_residual"] <= 1e-12, info
    assert rel_l2(out.core, alpha_o) <= 1e-10


# ------------------------------------------------------------------------------ full size
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "large_f32_reference.npz")


@pytest.mark.skipif(not __import__("os").path.exists(GOLDEN), reason="oracle reference not generated")
def test_full_size_against_oracle_reference(dev):
    # 2M FP32 points, ranks 24^3 (R = 13824), degree 31, M = 200,000 sampled rows: the launch
    # configuration of the benchmark.  The reference holds the oracle's model and its FP64
    # core of the sampled problem (tests/golden/make_large_golden.py, oracle only).
    ref = np.load(GOLDEN)
    w = datagen.large_f32()
    coefs = [ref[f"coefs{k}"] for k in range(3)]
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, ref["core0"], coefs)
    x, y, z, v = [D(a, dev) for a in w.soa()]
    idx = D(sample_without_replacement(w.seed, STREAM_LS, w.n, w.n_samples).astype(np.int32), dev)
    U, vs = fst.fst_factor_eval(gm, x, y, z, v, idx)
    # Gram entries against the oracle's: the diagonal and a seeded sample of 131,072
    # lower-triangle entries (uniform over the triangle, plus the whole 64 x 64 block in the
    # far corner), each route at the FP32 bar of 1e-5
    rows, cols = D(ref["gram_rows"].astype(np.int64), dev), D(ref["gram_cols"].astype(np.int64), dev)

    def check_gram(G):
        assert rel_l2(np.diag(H(G)), ref["gram_diag"]) <= 1e-5
        gs = H(G[rows, cols])
        assert rel_l2(gs, ref["gram_vals"]) <= 1e-5
        corner = slice(len(gs) - 4096, len(gs))
        assert rel_l2(gs[corner], ref["gram_vals"][corner]) <= 1e-5

    G, h = fst.fst_gram(gm, U, vs)                 # Khatri-Rao route (minimal workspace)
    assert rel_l2(H(h), ref["h"]) <= 1e-5
    check_gram(G)
    del G
    # the dense route as the benchmark times it: A^T of all M rows, then the dense Gram
    At, _ = fst.fst_design_rows(gm, U, Sp=(w.n_samples + 63) // 64 * 64)
    Gd, _ = fst.fst_gram_rows(At)
    del At
    check_gram(Gd)
    del Gd
    torch.cuda.empty_cache()
    # the split 16-bit Grams of the precision form
    for code in (fst.FST_GRAM_F16X2, fst.FST_GRAM_BF16X3):
        Gs, _ = fst.fst_gram(gm, U, gram_prec=code)
        check_gram(Gs)
        del Gs
        torch.cuda.empty_cache()
    alpha = ref["alpha"]
    # FP32 rows: kappa(G) ~ 6e7 amplifies FP32 rounding in the core; three FP64-residual
    # refinement steps bring it to the oracle's core
    out32 = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed, refine_steps=3)
    assert rel_l2(out32.core, alpha) <= 1e-6
    # the same with the workspace of the dense route
    ws = torch.empty(fst.fst_refit_workspace_bytes(gm, fst.FST_F32, w.n_samples, 3)
                     + fst.fst_gram_dense_workspace_bytes(gm, fst.FST_F32, w.n_samples), dtype=torch.uint8, device=dev)
    outd = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed, refine_steps=3, ws=ws)
    del ws
    torch.cuda.empty_cache()
    assert rel_l2(outd.core, alpha) <= 1e-6
    # the precision form as configured: split 16-bit Grams and three FP64-residual steps
    for code in (fst.FST_GRAM_F16X2, fst.FST_GRAM_BF16X3):
        outs = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed, gram_prec=code, refine_steps=3)
        assert outs.solve_info()["gram_prec"] == code
        assert rel_l2(outs.core, alpha) <= 1e-6
        del outs
        torch.cuda.empty_cache()
    # a single FP16 term needs more steps at this conditioning
    out16 = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed, gram_prec=fst.FST_GRAM_F16, refine_steps=9)
    assert rel_l2(out16.core, alpha) <= 1e-6
    # the FP16 Gram by the dense route (16-bit rows materialised), then the same refinement
    ws = torch.empty(fst.fst_refit_workspace_bytes(gm, fst.FST_F32, w.n_samples, 9)
                     + fst.fst_gram_dense_workspace_bytes(gm, fst.FST_F32, w.n_samples), dtype=torch.uint8, device=dev)
    out16d = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed, gram_prec=fst.FST_GRAM_F16, refine_steps=9,
                                ws=ws)
    del ws
    torch.cuda.empty_cache()
    assert rel_l2(out16d.core, alpha) <= 1e-6
    # reconstruction at sampled output points, against the oracle's field of its own core
    om = OModel(w.lo, w.hi, w.rank, w.degree, alpha.reshape(w.rank), coefs)
    f = H(fst.fst_eval(out32, x, y, z))
    pick = np.random.default_rng(0).choice(w.n, 20000, replace=False)
    fr = reconstruct.evaluate(om, w.pts[pick].astype(np.float64))
    assert rel_l2(f[pick], fr) <= 1e-5


# ------------------------------------------------------------------------------ outside the box
def _per_point_rel(a, b):
    """max over points of ||a_q - b_q|| / ||b_q|| (rows are points)."""
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


@pytest.mark.parametrize("rank,degree", [((24, 24, 24), (31, 31, 31)), ((16, 8, 5), (15, 7, 31))])
def test_factor_eval_outside_the_box(dev, rank, degree):
    """FP32 factor values at points up to three half-widths from the box centre (|t| <= 3): the
    basis grows like (|t| + sqrt(t^2 - 1))^m there, and the kernel scales each point's basis by
    its own power of two to keep its 16-bit terms in range.  The values match the oracle's to
    1e-5 (relative L2 over all points, whose size the farthest points set), and every point's
    values to 5e-5 relative to that point's own magnitude: a wrong scale for one point would
    show as an O(1) error there, while FP32 alone leaves t rounded by about 1e-6 at |t| <= 3,
    which the degree-31 basis amplifies up to m / sqrt(t^2 - 1) (about 1.1e-5 measured)."""
    om, gm = _models(5, rank, degree, lo=(0, 0, 0), hi=(4, 1, 1))
    pts = _pts(6, 6001, (-4, -1, -1), (8, 2, 2), np.float32)     # t in [-3, 3] in every mode
    x, y, z = _soa(pts, dev)
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    ref = lsq.factor_values(om, pts.astype(np.float64))
    Uh = H(U)
    off = 0
    for k in range(3):
        got = Uh[off:off + rank[k]].T.astype(np.float64)
        assert rel_l2(got, ref[k]) <= 1e-5, k
        assert _per_point_rel(got, ref[k]) <= 5e-5, k
        off += rank[k]


def test_eval_outside_the_box(dev):
    """FP32 reconstruction (eq. (1)) at points up to two half-widths out (|t| <= 2), where the
    factor values of a degree-15 model grow by up to 1e8: within 1e-5 of the oracle's field
    over the points inside the box and over those outside it."""
    rank, degree = (8, 12, 6), (15, 11, 13)
    om, gm = _models(7, rank, degree, lo=(0, 0, 0), hi=(4, 1, 1))
    pts = _pts(8, 20000, (-2, -0.5, -0.5), (6, 1.5, 1.5), np.float32)   # t in [-2, 2]
    x, y, z = _soa(pts, dev)
    out = torch.empty_like(x)
    fst.fst_eval(gm, x, y, z, out)
    f = H(out).astype(np.float64)
    ref = reconstruct.evaluate(om, pts.astype(np.float64))
    inside = np.all((pts >= (0, 0, 0)) & (pts <= (4, 1, 1)), axis=1)
    assert inside.sum() > 1000 and (~inside).sum() > 1000
    assert rel_l2(f[inside], ref[inside]) <= 1e-5
    assert rel_l2(f[~inside], ref[~inside]) <= 1e-5
