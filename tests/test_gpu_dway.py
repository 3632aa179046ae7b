"""GPU parity of the d-way calls (fst_eval_d, fst_refit_core_d) through the C ABI for 4-way
models (Sec. 2 format with d = 4; the space-time data of Sec. 6) against the oracle
(``oracle.reconstruct.evaluate``, ``oracle.lsq.refit_core``, pinned on the CPU), and for 3-way
models against the 3-way calls.

Tolerances (relative L2): FP64 1e-10.  FP32 1e-5 for reconstruction; for the refit, 1e-5 on
designs with orthonormal factor functions (kappa(G) of order 1-10, so FP32 rows and FP32 MFMA
with FP64 accumulation stay near 1e-6).
"""
import numpy as np
import pytest

from datagen import random_model_parts
from oracle.lsq import design_rows as lsq_design_rows, refit_core
from oracle.model import Model as OModel
from oracle.reconstruct import evaluate, rel_l2

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


def _models(seed, rank, degree, lo=None, hi=None, orthonormal=False):
    d = len(rank)
    lo = lo or (-1.0,) * d
    hi = hi or (1.0,) * d
    if orthonormal:
        rng = np.random.default_rng(seed)
        core = rng.standard_normal(tuple(rank))
        coefs = [np.linalg.qr(rng.standard_normal((degree[k] + 1, rank[k])))[0] for k in range(d)]
    else:
        core, coefs = random_model_parts(seed, rank, degree)
    return (OModel(tuple(lo), tuple(hi), tuple(rank), tuple(degree), core, coefs),
            fst.fst_model_from_parts(lo, hi, rank, degree, core, coefs))


def _points(seed, n, lo, hi, dtype):
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return (lo + (hi - lo) * rng.random((n, len(lo)))).astype(dtype)


# (ranks, degrees, n): ragged ranks and sizes; rank 1; degree 0 in a mode; rank-slice widths
# 4 .. 32 (the last two modes set the LDS slice); more (j1, j2) pairs than one 64 KB LDS slice
# holds (8 x 4 pairs of 32 x 30 FP64 entries: four slices)
EVAL_CASES = [
    ((3, 2, 4, 2), (5, 3, 6, 4), 3001),
    ((1, 1, 1, 1), (0, 2, 0, 3), 257),
    ((5, 6, 7, 9), (11, 17, 9, 20), 1000),
    ((2, 3, 13, 11), (20, 20, 31, 31), 777),
    ((8, 4, 32, 30), (31, 7, 31, 31), 600),
]


@pytest.mark.parametrize("rank,degree,n", EVAL_CASES)
def test_eval_d_four_way_fp64_matches_oracle(dev, rank, degree, n):
    print(f"eval4 fp64 rank={rank} degree={degree} n={n}", flush=True)
    lo, hi = (0.0, -2.0, 1.0, 0.0), (4.0, 1.0, 3.0, 10.0)
    om, gm = _models(sum(rank), rank, degree, lo, hi)
    pts = _points(n, n, lo, hi, np.float64)
    out = fst.fst_eval_d(gm, [D(pts[:, k], dev) for k in range(4)])
    assert rel_l2(out.cpu().numpy(), evaluate(om, pts)) <= 1e-10


@pytest.mark.parametrize("rank,degree,n", EVAL_CASES[:4])
def test_eval_d_four_way_fp32_matches_oracle(dev, rank, degree, n):
    print(f"eval4 fp32 rank={rank} degree={degree} n={n}", flush=True)
    lo, hi = (-1.0,) * 4, (1.0,) * 4
    om, gm = _models(7 + sum(rank), rank, degree, orthonormal=True)
    pts = _points(n + 1, n, lo, hi, np.float32)
    out = fst.fst_eval_d(gm, [D(pts[:, k], dev) for k in range(4)])
    assert rel_l2(out.cpu().numpy(), evaluate(om, pts.astype(np.float64))) <= 1e-5


def test_eval_d_many_rounds_and_empty(dev):
    # more points than one pass of the grid (2048 workgroups x 256 threads), and n = 0
    rank, degree = (2, 3, 2, 3), (4, 4, 4, 4)
    om, gm = _models(3, rank, degree, orthonormal=True)
    n = 600_001
    pts = _points(5, n, (-1.0,) * 4, (1.0,) * 4, np.float32)
    out = fst.fst_eval_d(gm, [D(pts[:, k], dev) for k in range(4)])
    assert rel_l2(out.cpu().numpy(), evaluate(om, pts.astype(np.float64))) <= 1e-5
    empty = [torch.empty(0, dtype=torch.float32, device=dev) for _ in range(4)]
    assert fst.fst_eval_d(gm, empty).numel() == 0


def test_eval_d_three_way_is_fst_eval(dev):
    om, gm = _models(4, (5, 4, 6), (9, 8, 7))
    pts = _points(6, 2000, (-1.0,) * 3, (1.0,) * 3, np.float64)
    c = [D(pts[:, k], dev) for k in range(3)]
    a = fst.fst_eval_d(gm, c)
    b = fst.fst_eval(gm, *c)
    assert torch.equal(a, b)


# refit: multi-chunk (M > 16384 rows, ragged last chunk) and single-chunk cases
@pytest.mark.parametrize("rank,degree,n,M", [
    ((3, 2, 4, 2), (5, 3, 6, 4), 60_000, 40_001),
    ((4, 3, 5, 6), (7, 7, 7, 7), 5_000, 1_500),
    ((2, 2, 9, 17), (9, 9, 12, 20), 20_000, 4_000),
])
def test_refit_d_four_way_fp64_matches_oracle(dev, rank, degree, n, M):
    print(f"refit4 fp64 rank={rank} n={n} M={M}", flush=True)
    lo, hi = (0.0, -1.0, 2.0, 0.0), (4.0, 1.0, 3.0, 1.0)
    om, gm = _models(11, rank, degree, lo, hi, orthonormal=True)
    pts = _points(12, n, lo, hi, np.float64)
    vals = evaluate(om, pts) + 0.1 * np.random.default_rng(13).standard_normal(n)
    alpha_o, _, _, _ = refit_core(om, pts, vals, M, seed=17)
    out = fst.fst_refit_core_d(gm, [D(pts[:, k], dev) for k in range(4)], D(vals, dev), M, 17)
    assert out.info()["d"] == 4 and out.core.shape == tuple(rank)
    assert rel_l2(out.core, alpha_o) <= 1e-10
    assert out.solve_info()["gram_prec"] == fst.FST_GRAM_F64


def test_refit_d_four_way_fp32_matches_oracle(dev):
    rank, degree, n, M = (4, 5, 3, 6), (9, 8, 7, 10), 50_000, 20_000
    print(f"refit4 fp32 rank={rank} n={n} M={M}", flush=True)
    om, gm = _models(21, rank, degree, orthonormal=True)
    pts = _points(22, n, (-1.0,) * 4, (1.0,) * 4, np.float32)
    vals = (evaluate(om, pts.astype(np.float64)) + 0.1 * np.random.default_rng(23).standard_normal(n)).astype(
        np.float32)
    alpha_o, _, _, _ = refit_core(om, pts.astype(np.float64), vals.astype(np.float64), M, seed=29)
    out = fst.fst_refit_core_d(gm, [D(pts[:, k], dev) for k in range(4)], D(vals, dev), M, 29)
    assert rel_l2(out.core, alpha_o) <= 1e-5
    assert out.solve_info()["gram_prec"] == fst.FST_GRAM_F32


def test_refit_d_three_way_matches_the_khatri_rao_refit(dev):
    rank, degree, n, M = (5, 4, 6), (8, 8, 8), 30_000, 20_000
    om, gm = _models(31, rank, degree, orthonormal=True)
    pts = _points(32, n, (-1.0,) * 3, (1.0,) * 3, np.float64)
    vals = evaluate(om, pts) + 0.05 * np.random.default_rng(33).standard_normal(n)
    c = [D(pts[:, k], dev) for k in range(3)]
    v = D(vals, dev)
    dense = fst.fst_refit_core_d(gm, c, v, M, 5)
    kr = fst.fst_refit_core(gm, *c, v, M, 5, gram_prec=fst.FST_GRAM_F64)
    assert rel_l2(dense.core, kr.core) <= 1e-10
    alpha_o, _, _, _ = refit_core(om, pts, vals, M, seed=5)
    assert rel_l2(dense.core, alpha_o) <= 1e-10


def test_refit_d_rejects_bad_arguments(dev):
    om, gm = _models(2, (2, 2, 2, 2), (3, 3, 3, 3))
    pts = _points(3, 500, (-1.0,) * 4, (1.0,) * 4, np.float64)
    c = [D(pts[:, k], dev) for k in range(4)]
    v = D(pts[:, 0], dev)
    for M in (16, 501):   # M <= R, M > n
        with pytest.raises(fst.FstError) as e:
            fst.fst_refit_core_d(gm, c, v, M, 1)
        assert e.value.status == fst.FST_E_INVAL
    _, g2 = _models(2, (5, 2, 2, 2), (3, 3, 3, 3))   # r_1 > p_1 + 1
    with pytest.raises(fst.FstError) as e:
        fst.fst_refit_core_d(g2, c, v, 100, 1)
    assert e.value.status == fst.FST_E_INVAL
    # 3-way calls refuse a 4-way model
    with pytest.raises(fst.FstError) as e:
        fst.fst_eval(gm, c[0], c[1], c[2])
    assert e.value.status == fst.FST_E_INVAL


def test_fit_d_four_way_end_to_end_fp64(dev):
    # Algorithm 1 (4-D interpolation, 4-way ST-HOSVD, sparse fits) + Algorithm 2 on the GPU,
    # against the oracle's pipeline on the same seeded space-time data
    import datagen
    from oracle import pipeline
    w = datagen.make_workload("t4", seed=8, n=20_000, n_gauss=6, grid=(8,) * 4, rank=(3, 3, 2, 2),
                              degree=(6,) * 4, interp_fraction=0.3, n_samples=3000, dtype=np.float64,
                              lo=(-1.0, -1.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0, 2.0))
    print("fit4 end to end", flush=True)
    mo = pipeline.fit(w.pts, w.vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction, w.n_samples, w.seed)
    p = fst.make_params_d(d=4, dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=w.grid, rank=w.rank, degree=w.degree,
                          interp_fraction=w.interp_fraction, n_samples=w.n_samples, seed=w.seed)
    c = [D(a, dev) for a in w.soa()]
    gm = fst.fst_fit_d(p, c[:4], c[4])
    for k in range(4):
        np.testing.assert_array_equal(gm.coefs(k) != 0, mo.coefs[k] != 0)
        assert rel_l2(gm.coefs(k), mo.coefs[k]) <= 1e-10
    print(f"core rel-L2 {rel_l2(gm.core, mo.core):.3e}", flush=True)
    assert rel_l2(gm.core, mo.core) <= 1e-10
    f = fst.fst_eval_d(gm, c[:4]).cpu().numpy()
    err_gpu, err_ref = rel_l2(f, w.vals), rel_l2(evaluate(mo, w.pts), w.vals)
    assert abs(err_gpu - err_ref) <= 1e-10 * err_ref


def test_fit_d_four_way_fp32_ranks_from_precision(dev):
    import datagen
    from oracle import pipeline
    from oracle.sthosvd import ranks_for_precision
    w = datagen.make_workload("t4", seed=9, n=40_000, n_gauss=6, grid=(8,) * 4, rank=(6,) * 4,
                              degree=(7,) * 4, interp_fraction=0.3, n_samples=8000, dtype=np.float32,
                              lo=(-1.0, -1.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0, 2.0))
    eps = 0.2
    T = pipeline.compress(w.pts.astype(np.float64), w.vals.astype(np.float64), w.lo, w.hi, w.grid, (1,) * 4,
                          w.degree, w.interp_fraction, w.seed).info["grid_tensor"]
    r = tuple(min(a, 6) for a in ranks_for_precision(T, eps))
    print(f"fit4 fp32 eps={eps} ranks={r}", flush=True)
    p = fst.make_params_d(d=4, dtype=fst.FST_F32, lo=w.lo, hi=w.hi, grid=w.grid, rank=w.rank, degree=w.degree,
                          interp_fraction=w.interp_fraction, n_samples=w.n_samples, seed=w.seed, eps=eps)
    c = [D(a, dev) for a in w.soa()]
    gm = fst.fst_fit_d(p, c[:4], c[4])
    assert gm.info()["rank"] == r
    mo = pipeline.fit(w.pts.astype(np.float64), w.vals.astype(np.float64), w.lo, w.hi, w.grid, r, w.degree,
                      w.interp_fraction, w.n_samples, w.seed)
    # FP32 rows and FP32 sums in the Gram, no refinement: ||d alpha|| / ||alpha|| is bounded by
    # kappa(G) times the relative Gram error, a small multiple of 2^-24
    from oracle import lsq
    _, _, G, _ = lsq.refit_core(mo, w.pts.astype(np.float64), w.vals.astype(np.float64), w.n_samples, w.seed)
    kappa = np.linalg.cond(G)
    err = rel_l2(gm.core, mo.core)
    print(f"fp32 4-way core rel-L2 {err:.3e}, kappa(G) {kappa:.3e}", flush=True)
    assert err <= max(1e-6, 8 * kappa * 2.0 ** -24)


# ------------------------------------------------------------------------------ dense route calls
# 3-way rows whose count is a multiple of 4 take the vector kernel (4 FP32 or 2 FP64 rows per
# thread), the others the scalar one; both with a padded tail
@pytest.mark.parametrize("rank,mrows,Sp", [((3, 2, 4, 2), 1000, 1024), ((5, 6, 7, 9), 777, 832),
                                           ((4, 3, 5), 130, 192), ((1, 1, 1, 1), 1, 64),
                                           ((6, 5, 4, 17), 4097, 4160), ((4, 3, 5), 1000, 1024),
                                           ((7, 6, 5), 4100, 4160), ((2, 1, 3), 4, 64)])
def test_design_rows_and_gram_rows(dev, rank, mrows, Sp):
    # the design rows of eq. (6) from arbitrary factor values: the kernel forms the products in
    # the oracle's order, so FP64 rows are bit-exact; then G and h from the rows in two chunks
    print(f"design rows rank={rank} mrows={mrows} Sp={Sp}", flush=True)
    rng = np.random.default_rng(sum(rank) + mrows)
    Uk = [rng.standard_normal((mrows, r)) for r in rank]
    vs = rng.standard_normal(mrows)
    A = lsq_design_rows(Uk)
    R = A.shape[1]
    m = _models(3, rank, tuple(r + 1 for r in rank))[1]
    for dtype in (np.float64, np.float32):
        U = D(np.concatenate([u.T for u in Uk]).astype(dtype), dev)
        At, b = fst.fst_design_rows(m, U, D(vs.astype(dtype), dev), Sp=Sp)
        At_h, b_h = At.cpu().numpy(), b.cpu().numpy()
        assert At_h.shape == (R, Sp)
        assert np.all(At_h[:, mrows:] == 0) and np.all(b_h[mrows:] == 0)
        if dtype == np.float64:
            np.testing.assert_array_equal(At_h[:, :mrows], A.T)
        else:
            A32 = lsq_design_rows([u.astype(np.float32).astype(np.float64) for u in Uk])
            assert rel_l2(At_h[:, :mrows], A32.T) <= 1e-6
        np.testing.assert_array_equal(b_h[:mrows], vs.astype(dtype))
        Ah = At_h[:, :mrows].astype(np.float64)
        Gr, hr = Ah @ Ah.T, Ah @ b_h[:mrows].astype(np.float64)
        tol = 1e-12 if dtype == np.float64 else 1e-6
        G, h = fst.fst_gram_rows(At, b)
        low = np.tril_indices(R)
        assert rel_l2(G.cpu().numpy()[low], Gr[low]) <= tol and rel_l2(h.cpu().numpy(), hr) <= tol
        assert np.all(np.triu(G.cpu().numpy(), 1) == 0)          # strictly upper part untouched
        if Sp >= 128:   # the same sums over two column chunks of At, the second accumulated
            c = Sp // 128 * 64
            G2, h2 = fst.fst_gram_rows(At[:, :c].contiguous(), b[:c].contiguous())
            fst.fst_gram_rows(At[:, c:].contiguous(), b[c:].contiguous(), G=G2, h=h2, accumulate=True)
            assert rel_l2(G2.cpu().numpy()[low], Gr[low]) <= tol and rel_l2(h2.cpu().numpy(), hr) <= tol


def test_design_and_gram_rows_reject_bad_sizes(dev):
    m = _models(3, (3, 2, 4), (4, 4, 4))[1]
    U = torch.zeros((9, 100), dtype=torch.float64, device=dev)
    for Sp in (96, 64):                      # not a multiple of 64; fewer than mrows
        with pytest.raises(fst.FstError) as e:
            fst.fst_design_rows(m, U, Sp=Sp, At=torch.empty((24, 128), dtype=torch.float64, device=dev))
        assert e.value.status == fst.FST_E_INVAL
    At = torch.zeros((24, 100), dtype=torch.float64, device=dev)
    with pytest.raises(fst.FstError) as e:
        fst.fst_gram_rows(At)
    assert e.value.status == fst.FST_E_INVAL
