"""CPU tests of the C-ABI library: every declared symbol is exported, the host steps of
Algorithm 1 match the oracle, models round-trip through serialisation, and bad arguments
are rejected with the documented status codes.  No GPU is touched."""
import ctypes
import os
import re

import numpy as np
import pytest

import datagen
from oracle import interp, pipeline, sampler, sparsefit, sthosvd
from oracle.basis import legendre_orthonormal
from oracle.model import Model as OModel
from oracle.reconstruct import rel_l2
from oracle.sthosvd import ranks_for_precision, st_hosvd, tucker_full

fst = pytest.importorskip("paper_1907_05884_amd.binding")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "fst.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fst_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = ctypes.CDLL(fst.LIB_PATH)
    declared = _declared_symbols()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(fst.EXPORTED_SYMBOLS)


def test_params_struct_layout_matches():
    p = fst.make_params()
    assert p.struct_size == ctypes.sizeof(fst.fst_fit_params)
    assert fst.fst_version().startswith("fst-mi355x")


@pytest.mark.parametrize("seed,stream,n,m", [(1, 2, 2000, 500), (7, 1, 100000, 5000), (3, 2, 17, 17), (3, 2, 5, 0)])
def test_sampler_bit_exact_with_oracle(seed, stream, n, m):
    np.testing.assert_array_equal(fst.fst_sample_indices(seed, stream, n, m),
                                  sampler.sample_without_replacement(seed, stream, n, m))


def test_idw_matches_oracle():
    rng = np.random.default_rng(0)
    xi = rng.uniform(-1, 1, (3000, 3))
    v = rng.standard_normal(3000)
    grid = (9, 12, 7)
    ref = interp.idw_to_grid(xi, v, grid)
    got = fst.fst_idw_grid(xi, v, grid, k=8, power=2.0)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)
    # exact hit on a grid node takes the point's value
    xi2 = np.vstack([xi, interp.grid_points(grid)[[5]]])
    v2 = np.concatenate([v, [42.0]])
    assert fst.fst_idw_grid(xi2, v2, grid).reshape(-1)[5] == 42.0
    # fewer points than neighbours, and a different power
    np.testing.assert_allclose(fst.fst_idw_grid(xi[:5], v[:5], (4, 4, 4), k=8, power=3.0),
                               interp.idw_to_grid(xi[:5], v[:5], (4, 4, 4), k=8, power=3.0),
                               rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("dims,rank", [((12, 10, 9), (4, 3, 2)), ((20, 6, 7), (5, 6, 7)), ((16, 16, 16), (3, 3, 3))])
def test_sthosvd_matches_oracle(dims, rank):
    rng = np.random.default_rng(sum(dims))
    T = rng.standard_normal(dims)
    core_o, W_o, s_o = sthosvd.st_hosvd(T, rank)
    core, W, S = fst.fst_sthosvd(T, rank)
    for k in range(3):
        np.testing.assert_allclose(W[k], W_o[k], atol=1e-10)
        np.testing.assert_allclose(S[k][: len(s_o[k])], s_o[k], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(core, core_o, atol=1e-10)


def test_sthosvd_exact_low_rank_recovery():
    rng = np.random.default_rng(9)
    r = (3, 4, 2)
    G = rng.standard_normal(r)
    Q = [np.linalg.qr(rng.standard_normal((n, k)))[0] for n, k in zip((14, 11, 10), r)]
    X = sthosvd.tucker_full(G, Q)
    core, W, _ = fst.fst_sthosvd(X, r)
    assert np.linalg.norm(sthosvd.tucker_full(core, W) - X) / np.linalg.norm(X) < 1e-13


def test_sparse_fit_matches_oracle():
    nodes = interp.grid_nodes(32)
    rng = np.random.default_rng(1)
    Phi = legendre_orthonormal(nodes, 15)
    c = np.zeros((16, 4))
    c[[0, 3, 7], 0] = [1.0, -0.5, 0.25]
    c[[2], 1] = [2.0]
    W = Phi @ c
    W[:, 2] = np.sin(3 * nodes)
    W[:, 3] = np.exp(-nodes ** 2) + 1e-3 * rng.standard_normal(32)
    ref = sparsefit.fit_factor(W, nodes, 15)
    got = fst.fst_sparse_fit(W, 15)
    np.testing.assert_array_equal(got != 0, ref != 0)      # identical supports
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(got[:, :2], c[:, :2], atol=1e-12)


def test_compress_host_matches_oracle_small():
    w = datagen.small_f64(n=6000, n_samples=1500)
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=(16, 16, 16), rank=(5, 4, 3),
                        degree=(9, 9, 9), interp_fraction=0.2, n_samples=1500, seed=w.seed)
    x, y, z, v = w.soa()
    m = fst.fst_compress_host(p, x, y, z, v)
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, (16, 16, 16), (5, 4, 3), (9, 9, 9), 0.2, w.seed)
    assert rel_l2(m.core, mo.core) <= 1e-10
    for k in range(3):
        Ck, Co = m.coefs(k), mo.coefs[k]
        np.testing.assert_array_equal(Ck != 0, Co != 0)
        assert rel_l2(Ck, Co) <= 1e-10


def _decaying_tensor(seed, dims, core_dims):
    # full multilinear rank core_dims with entries decaying like 10^(-(a+b+c)/3), rotated by
    # random orthonormal factors: the singular values of every unfolding decay steadily
    rng = np.random.default_rng(seed)
    a, b, c = np.meshgrid(*[np.arange(n) for n in core_dims], indexing="ij")
    G = rng.standard_normal(core_dims) * 10.0 ** (-(a + b + c) / 3.0)
    Q = [np.linalg.qr(rng.standard_normal((n, n)))[0][:, :m] for n, m in zip(dims, core_dims)]
    return tucker_full(G, Q)


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 3e-3, 1e-6])
def test_sthosvd_eps_matches_oracle_and_meets_precision(eps):
    # ranks from the precision (Sec. 4.1, Table 1): the library's rule against the oracle's,
    # the decomposition at those ranks against the oracle's, and ||T - T~|| <= eps ||T||
    T = _decaying_tensor(0, (20, 18, 16), (10, 9, 7))
    r, core, W, _ = fst.fst_sthosvd_eps(T, eps, (20, 18, 16))
    assert r == ranks_for_precision(T, eps)
    c_o, W_o, _ = st_hosvd(T, r)
    np.testing.assert_allclose(core, c_o, atol=1e-10)
    for k in range(3):
        np.testing.assert_allclose(W[k], W_o[k], atol=1e-10)
    assert np.linalg.norm(T - tucker_full(core, W)) <= eps * np.linalg.norm(T) * (1 + 1e-12)


def test_sthosvd_eps_caps_and_errors():
    T = _decaying_tensor(1, (12, 11, 10), (8, 8, 8))
    r, core, W, _ = fst.fst_sthosvd_eps(T, 1e-8, (4, 5, 3))
    assert r == (4, 5, 3)
    c_o, _, _ = st_hosvd(T, r)
    np.testing.assert_allclose(core, c_o, atol=1e-10)
    for bad in (0.0, 1.0, -1e-3):
        with pytest.raises(fst.FstError):
            fst.fst_sthosvd_eps(T, bad, (4, 4, 4))


def test_compress_host_with_eps_ranks_matches_oracle():
    # Algorithm 1 with ranks from the precision: the ranks the oracle's rule picks on the
    # oracle's interpolated grid (identical to the library's grid), capped by rank[]
    w = datagen.small_f64(n=6000, n_samples=1500)
    grid, degree, caps, eps = (16, 16, 16), (11, 11, 11), (10, 10, 10), 0.1
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=grid, rank=caps, degree=degree,
                        interp_fraction=0.2, n_samples=1500, seed=w.seed, eps=eps)
    m = fst.fst_compress_host(p, *w.soa())
    T = pipeline.compress(w.pts, w.vals, w.lo, w.hi, grid, (1, 1, 1), degree, 0.2, w.seed).info["grid_tensor"]
    r = ranks_for_precision(T, eps)
    assert all(1 <= r[k] <= caps[k] for k in range(3)) and all(r[k] <= r[(k + 1) % 3] * r[(k + 2) % 3] for k in range(3))
    assert m.info()["rank"] == r
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, grid, r, degree, 0.2, w.seed)
    assert rel_l2(m.core, mo.core) <= 1e-10


def test_model_parts_roundtrip_and_serialisation():
    core, coefs = datagen.random_model_parts(3, (4, 3, 5), (6, 7, 5))
    m = fst.fst_model_from_parts((0, 0, 0), (4, 1, 1), (4, 3, 5), (6, 7, 5), core, coefs)
    np.testing.assert_array_equal(m.core, core)
    for k in range(3):
        np.testing.assert_array_equal(m.coefs(k), coefs[k])
    inf = m.info()
    assert inf["rank"] == (4, 3, 5) and inf["degree"] == (6, 7, 5) and inf["hi"] == (4.0, 1.0, 1.0)
    om = OModel((0, 0, 0), (4, 1, 1), (4, 3, 5), (6, 7, 5), core, coefs)
    assert m.paper_bytes() == om.paper_bytes()
    blob = fst.fst_model_save(m)
    m2 = fst.fst_model_load(blob)
    np.testing.assert_array_equal(m2.core, core)
    for k in range(3):
        np.testing.assert_array_equal(m2.coefs(k), coefs[k])
    assert fst.fst_model_save(m2) == blob
    # truncated, corrupted and foreign buffers are rejected
    for bad in (blob[:-3], blob[:20], b"XXXX" + blob[4:], blob[:40] + bytes([blob[40] ^ 1]) + blob[41:]):
        with pytest.raises(fst.FstError) as e:
            fst.fst_model_load(bad)
        assert e.value.status == fst.FST_E_FORMAT


def test_invalid_arguments_are_rejected():
    core, coefs = datagen.random_model_parts(1, (2, 2, 2), (3, 3, 3))
    with pytest.raises(fst.FstError) as e:
        fst.fst_model_from_parts((0, 0, 0), (0, 1, 1), (2, 2, 2), (3, 3, 3), core, coefs)
    assert e.value.status == fst.FST_E_INVAL
    with pytest.raises(fst.FstError) as e:
        fst.fst_model_from_parts((0, 0, 0), (1, 1, 1), (40, 2, 2), (3, 3, 3), np.zeros(160),
                                 [np.zeros((4, 40)), coefs[1], coefs[2]])
    assert e.value.status == fst.FST_E_UNSUPPORTED
    bad = coefs[0].copy()
    bad[0, 0] = np.nan
    with pytest.raises(fst.FstError):
        fst.fst_model_from_parts((0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 3, 3), core, [bad, coefs[1], coefs[2]])
    x = np.zeros(100)
    # M <= R (Algorithm 2 needs S > R)
    p = fst.make_params(rank=(4, 4, 4), grid=(8, 8, 8), degree=(3, 3, 3), n_samples=64)
    with pytest.raises(fst.FstError) as e:
        fst.fst_fit_workspace_bytes(p, 100)
    assert e.value.status == fst.FST_E_INVAL
    # more factor functions than basis functions in a mode: the design rows are dependent
    p = fst.make_params(rank=(5, 4, 4), grid=(8, 8, 8), degree=(3, 3, 3), n_samples=200)
    with pytest.raises(fst.FstError, match="degree \\+ 1") as e:
        fst.fst_fit_workspace_bytes(p, 1000)
    assert e.value.status == fst.FST_E_INVAL
    # rank larger than the grid, rank larger than the product of the others
    for kw in (dict(rank=(9, 8, 8), grid=(8, 8, 8)), dict(rank=(2, 2, 5), grid=(8, 8, 8))):
        p = fst.make_params(degree=(3, 3, 3), n_samples=90, **kw)
        with pytest.raises(fst.FstError):
            fst.fst_compress_host(p, x, x, x, x)
    # non-finite data in the interpolation subset
    p = fst.make_params(rank=(2, 2, 2), grid=(6, 6, 6), degree=(3, 3, 3), n_samples=50, interp_fraction=1.0)
    xb = np.random.default_rng(0).uniform(-1, 1, 100)
    vb = xb.copy()
    vb[10] = np.inf
    with pytest.raises(fst.FstError) as e:
        fst.fst_compress_host(p, xb, xb, xb, vb)
    assert e.value.status == fst.FST_E_INVAL
    with pytest.raises(fst.FstError):
        fst.fst_sample_indices(1, 2, 10, 11)
    p.struct_size = 8
    with pytest.raises(fst.FstError):
        fst.fst_fit_workspace_bytes(p, 100)


def _model4(seed=1, rank=(3, 2, 4, 2), degree=(5, 3, 6, 4)):
    core, coefs = datagen.random_model_parts(seed, rank, degree)
    lo, hi = (0.0, -1.0, 2.0, 0.0), (4.0, 1.0, 3.0, 10.0)
    return OModel(lo, hi, rank, degree, core, coefs), fst.fst_model_from_parts(lo, hi, rank, degree, core, coefs)


def test_four_way_model_parts_info_and_serialisation():
    om, m = _model4()
    inf = m.info()
    assert inf["d"] == 4 and inf["rank"] == om.rank and inf["degree"] == om.degree
    assert inf["lo"] == om.lo and inf["hi"] == om.hi
    assert inf["nnz"] == om.nnz() and m.R == om.R
    np.testing.assert_array_equal(m.core, om.core)
    for k in range(4):
        np.testing.assert_array_equal(m.coefs(k), om.coefs[k])
    assert m.paper_bytes() == om.paper_bytes()
    blob = fst.fst_model_save(m)
    m2 = fst.fst_model_load(blob)
    assert m2.info() == inf
    np.testing.assert_array_equal(m2.core, om.core)
    for k in range(4):
        np.testing.assert_array_equal(m2.coefs(k), om.coefs[k])
    assert fst.fst_model_save(m2) == blob
    # a 3-way model built through the d-way constructor is the 3-way model
    core3, coefs3 = datagen.random_model_parts(2, (3, 4, 2), (5, 4, 6))
    lo3, hi3 = (-1.0,) * 3, (1.0,) * 3
    a = fst.fst_model_from_parts(lo3, hi3, (3, 4, 2), (5, 4, 6), core3, coefs3)
    cs = [np.ascontiguousarray(c) for c in coefs3]
    arr = (ctypes.c_void_p * 3)(*[c.ctypes.data_as(ctypes.c_void_p) for c in cs])
    h = ctypes.c_void_p()
    c3 = np.ascontiguousarray(core3)
    st = fst._fn["fst_model_from_parts_d"](3, np.asarray(lo3).ctypes.data_as(ctypes.c_void_p),
                                           np.asarray(hi3).ctypes.data_as(ctypes.c_void_p),
                                           np.asarray((3, 4, 2), np.int32).ctypes.data_as(ctypes.c_void_p),
                                           np.asarray((5, 4, 6), np.int32).ctypes.data_as(ctypes.c_void_p),
                                           c3.ctypes.data_as(ctypes.c_void_p), arr, ctypes.byref(h))
    assert st == fst.FST_OK
    b = fst.Model(h)
    assert fst.fst_model_save(a) == fst.fst_model_save(b)
    assert b.info()["d"] == 3


def test_three_way_calls_reject_four_way_models():
    om, m = _model4()
    st = fst._fn["fst_eval"](m.handle, fst.FST_F64, 10, None, None, None, None, None)
    assert st == fst.FST_E_INVAL and "3-way" in fst.fst_last_error()
    lo, hi = (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    rk, dg = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)()
    assert fst._fn["fst_model_info"](m.handle, lo, hi, rk, dg, None) == fst.FST_E_INVAL
    assert fst._fn["fst_refit_workspace_bytes"](m.handle, fst.FST_F32, 1000, 0) == 0
    assert fst._fn["fst_eval_grid_workspace_bytes"](m.handle, fst.FST_F32, 4, 4, 4) == 0
    assert fst._fn["fst_gram_workspace_bytes"](m.handle, 1000) == 0
    assert fst._fn["fst_refit_core_mixed_workspace_bytes"](m.handle, fst.FST_F32, 5000, 1000) == 0
    # the d-way workspace holds at least the FP64 Gram and the rows of one chunk
    ws = fst.fst_refit_core_d_workspace_bytes(m, fst.FST_F32, 1000)
    assert ws >= 8 * om.R * om.R + 4 * om.R * 1024
    # mode index bounds follow d
    out = np.empty((7, 2))
    assert fst._fn["fst_model_coefs"](m.handle, 3, out.ctypes.data_as(ctypes.c_void_p)) == fst.FST_OK
    assert fst._fn["fst_model_coefs"](m.handle, 4, out.ctypes.data_as(ctypes.c_void_p)) == fst.FST_E_INVAL
    # only d = 3 and d = 4 exist
    one = np.ones(5)
    ip = np.ones(5, np.int32)
    arr = (ctypes.c_void_p * 5)(*[one.ctypes.data_as(ctypes.c_void_p)] * 5)
    h = ctypes.c_void_p()
    st = fst._fn["fst_model_from_parts_d"](5, one.ctypes.data_as(ctypes.c_void_p),
                                           (one * 2).ctypes.data_as(ctypes.c_void_p),
                                           ip.ctypes.data_as(ctypes.c_void_p),
                                           (ip * 0).ctypes.data_as(ctypes.c_void_p),
                                           one.ctypes.data_as(ctypes.c_void_p), arr, ctypes.byref(h))
    assert st == fst.FST_E_UNSUPPORTED
    # the d-way calls reject a null coordinate list before touching the device
    st = fst._fn["fst_eval_d"](m.handle, fst.FST_F64, 10, None, None, None)
    assert st == fst.FST_E_INVAL


def _workload4(n=6000, seed=8):
    return datagen.make_workload("t4", seed=seed, n=n, n_gauss=6, grid=(8,) * 4, rank=(3, 3, 2, 2),
                                 degree=(6,) * 4, interp_fraction=0.3, n_samples=1000, dtype=np.float64,
                                 lo=(-1.0, -1.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0, 2.0))


def test_idw_four_dimensional_matches_oracle():
    # the library's 4-D inverse-distance grid against the oracle's (exact kNN by a k-d tree),
    # through Algorithm 1's grid tensor
    w = _workload4()
    grid = (6, 7, 5, 8)
    p = fst.make_params_d(d=4, dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=grid, rank=(1, 1, 1, 1),
                          degree=(3,) * 4, interp_fraction=0.3, n_samples=1000, seed=w.seed)
    coords, v = w.soa()[:4], w.soa()[4]
    m = fst.fst_compress_host_d(p, coords, v)
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, grid, (1, 1, 1, 1), (3,) * 4, 0.3, w.seed)
    # rank (1,1,1,1): the core is the projection of the grid tensor on the leading singular
    # vectors, so equal cores need equal grid tensors up to rounding
    np.testing.assert_allclose(m.core, mo.core, rtol=1e-10)
    T = mo.info["grid_tensor"]
    assert T.shape == grid and np.isfinite(T).all()


def test_compress_host_d_matches_oracle_four_way():
    w = _workload4()
    grid, rank, degree = (8, 8, 8, 8), (3, 3, 2, 2), (6, 6, 6, 6)
    p = fst.make_params_d(d=4, dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=grid, rank=rank, degree=degree,
                          interp_fraction=0.3, n_samples=1000, seed=w.seed)
    coords, v = w.soa()[:4], w.soa()[4]
    m = fst.fst_compress_host_d(p, coords, v)
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, grid, rank, degree, 0.3, w.seed)
    assert m.info()["d"] == 4 and m.info()["rank"] == rank
    assert rel_l2(m.core, mo.core) <= 1e-10
    for k in range(4):
        Ck, Co = m.coefs(k), mo.coefs[k]
        np.testing.assert_array_equal(Ck != 0, Co != 0)
        assert rel_l2(Ck, Co) <= 1e-10


def test_compress_host_d_with_eps_ranks_matches_oracle():
    w = _workload4()
    grid, degree, caps, eps = (8, 8, 8, 8), (6, 6, 6, 6), (6, 6, 6, 6), 0.2
    p = fst.make_params_d(d=4, dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=grid, rank=caps, degree=degree,
                          interp_fraction=0.3, n_samples=2000, seed=w.seed, eps=eps)
    m = fst.fst_compress_host_d(p, w.soa()[:4], w.soa()[4])
    T = pipeline.compress(w.pts, w.vals, w.lo, w.hi, grid, (1,) * 4, degree, 0.3, w.seed).info["grid_tensor"]
    r = ranks_for_precision(T, eps)
    assert all(1 <= r[k] <= caps[k] for k in range(4)), r
    assert m.info()["rank"] == r
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, grid, r, degree, 0.3, w.seed)
    assert rel_l2(m.core, mo.core) <= 1e-10
    Tt = tucker_full(mo.core, mo.info["factors"])
    assert np.linalg.norm(T - Tt) <= eps * np.linalg.norm(T) * (1 + 1e-9)


def test_compress_host_d_three_way_is_the_three_way_compress():
    w = datagen.small_f64(n=6000, n_samples=1500)
    grid, rank, degree = (16, 16, 16), (5, 4, 3), (9, 9, 9)
    p3 = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=grid, rank=rank, degree=degree,
                         interp_fraction=0.2, n_samples=1500, seed=w.seed)
    pd = fst.make_params_d(d=3, dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=grid, rank=rank, degree=degree,
                           interp_fraction=0.2, n_samples=1500, seed=w.seed)
    x, y, z, v = w.soa()
    a = fst.fst_compress_host(p3, x, y, z, v)
    b = fst.fst_compress_host_d(pd, (x, y, z), v)
    assert fst.fst_model_save(a) == fst.fst_model_save(b)


def test_fit_params_d_validation():
    ok = dict(d=4, dtype=fst.FST_F64, grid=(8,) * 4, rank=(2,) * 4, degree=(5,) * 4, n_samples=100)
    assert fst.fst_fit_d_workspace_bytes(fst.make_params_d(**ok), 1000) > 0
    for bad, status in [(dict(rank=(9, 2, 2, 2)), fst.FST_E_INVAL),          # rank > grid
                        (dict(rank=(7, 1, 1, 1), grid=(8,) * 4), fst.FST_E_INVAL),  # rank > product of others
                        (dict(n_samples=16), fst.FST_E_INVAL),               # M <= R
                        (dict(degree=(40,) * 4), fst.FST_E_UNSUPPORTED)]:
        p = fst.make_params_d(**{**ok, **bad})
        assert fst._fn["fst_fit_d_workspace_bytes"](ctypes.byref(p), 1000) == 0
    p = fst.make_params_d(**ok)
    p.d = 5
    h = ctypes.c_void_p()
    assert fst._fn["fst_compress_host_d"](ctypes.byref(p), 10, None, None, ctypes.byref(h)) == fst.FST_E_UNSUPPORTED


def test_sparse_fit_lars_matches_oracle():
    nodes = interp.grid_nodes(32)
    rng = np.random.default_rng(1)
    Phi = legendre_orthonormal(nodes, 15)
    c = np.zeros((16, 5))
    c[[0, 3, 7], 0] = [1.0, -0.5, 0.25]
    c[[2], 1] = [2.0]
    W = Phi @ c
    W[:, 2] = np.sin(3 * nodes)
    W[:, 3] = np.exp(-nodes ** 2) + 1e-3 * rng.standard_normal(32)
    W[:, 4] = np.tanh(8 * nodes) + 1e-2 * rng.standard_normal(32)
    ref = sparsefit.fit_factor(W, nodes, 15, solver="lars")
    got = fst.fst_sparse_fit(W, 15, solver=fst.FST_SOLVER_LARS)
    np.testing.assert_array_equal(got != 0, ref != 0)      # identical supports
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(got[:, :2], c[:, :2], atol=1e-12)


def test_sparse_fit_lars_on_singular_vectors_matches_oracle():
    # the factor matrices of Algorithm 1 on the small workload: real singular vectors
    w = datagen.small_f64(n=6000, n_samples=1500)
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, (16, 16, 16), (6, 5, 4), (9, 9, 9), 0.2, w.seed)
    for k in range(3):
        Wk = mo.info["factors"][k]
        ref = sparsefit.fit_factor(Wk, interp.grid_nodes(16), 9, solver="lars")
        got = fst.fst_sparse_fit(Wk, 9, solver=fst.FST_SOLVER_LARS)
        np.testing.assert_array_equal(got != 0, ref != 0)
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-13)


def test_compress_host_with_lars_matches_oracle():
    w = datagen.small_f64(n=6000, n_samples=1500)
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=(16, 16, 16), rank=(5, 4, 3),
                        degree=(9, 9, 9), interp_fraction=0.2, n_samples=1500, seed=w.seed,
                        sparse_solver=fst.FST_SOLVER_LARS)
    m = fst.fst_compress_host(p, *w.soa())
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, (16, 16, 16), (5, 4, 3), (9, 9, 9), 0.2, w.seed,
                           solver="lars")
    assert rel_l2(m.core, mo.core) <= 1e-10
    for k in range(3):
        np.testing.assert_array_equal(m.coefs(k) != 0, mo.coefs[k] != 0)
        assert rel_l2(m.coefs(k), mo.coefs[k]) <= 1e-10
    # the 4-way compress takes the same solver
    w4 = _workload4()
    p4 = fst.make_params_d(d=4, dtype=fst.FST_F64, lo=w4.lo, hi=w4.hi, grid=(8,) * 4, rank=(3, 3, 2, 2),
                           degree=(6,) * 4, interp_fraction=0.3, n_samples=1000, seed=w4.seed,
                           sparse_solver=fst.FST_SOLVER_LARS)
    m4 = fst.fst_compress_host_d(p4, w4.soa()[:4], w4.soa()[4])
    mo4 = pipeline.compress(w4.pts, w4.vals, w4.lo, w4.hi, (8,) * 4, (3, 3, 2, 2), (6,) * 4, 0.3, w4.seed,
                            solver="lars")
    for k in range(4):
        np.testing.assert_array_equal(m4.coefs(k) != 0, mo4.coefs[k] != 0)
        assert rel_l2(m4.coefs(k), mo4.coefs[k]) <= 1e-10
    bad = fst.make_params(sparse_solver=7)
    assert fst._fn["fst_fit_workspace_bytes"](ctypes.byref(bad), 10000) == 0


@pytest.mark.parametrize("solver", ["omp", "lars"])
@pytest.mark.parametrize("s,q", [(3, 2), (2, 5), (4, 1)])
def test_sparse_fit_choice_matches_oracle(solver, s, q):
    nodes = interp.grid_nodes(48)
    rng = np.random.default_rng(s * 10 + q)
    # (|t - 0.1| carries noise: exactly piecewise linear, its PRESS path has steps of equal
    # PRESS to rounding, where either support is a valid answer)
    W = np.stack([1 + nodes - 0.5 * nodes ** 3, np.where(nodes < 0.25, -1.0, 2.0),
                  np.exp(-nodes ** 2) + 1e-3 * rng.standard_normal(48),
                  np.abs(nodes - 0.1) + 1e-3 * rng.standard_normal(48), np.sin(9 * nodes)], axis=1)
    p = 11
    ref = sparsefit.fit_factor_choice(W, nodes, p, s, q, solver=solver)
    code = fst.FST_SOLVER_LARS if solver == "lars" else fst.FST_SOLVER_OMP
    got = fst.fst_sparse_fit_choice(W, p, s, q, solver=code)
    np.testing.assert_array_equal(got != 0, ref != 0)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-13)
    assert np.any(got[p + 1:] != 0)          # some column keeps the wavelet fit


def test_compress_host_with_wavelets_matches_oracle():
    w = datagen.small_f64(n=6000, n_samples=1500)
    grid, rank, degree, wav = (16, 16, 16), (6, 5, 4), (9, 9, 9), (2, 3)
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=grid, rank=rank, degree=degree,
                        interp_fraction=0.2, n_samples=1500, seed=w.seed, wavelet=wav)
    m = fst.fst_compress_host(p, *w.soa())
    mo = pipeline.compress(w.pts, w.vals, w.lo, w.hi, grid, rank, degree, 0.2, w.seed, wavelet=wav)
    assert m.wavelets() == ((2, 3),) * 3
    assert rel_l2(m.core, mo.core) <= 1e-10
    for k in range(3):
        np.testing.assert_array_equal(m.coefs(k) != 0, mo.coefs[k] != 0)
        assert rel_l2(m.coefs(k), mo.coefs[k]) <= 1e-10
    assert m.paper_bytes() == mo.paper_bytes()
    blob = fst.fst_model_save(m)
    m2 = fst.fst_model_load(blob)
    assert m2.wavelets() == m.wavelets() and fst.fst_model_save(m2) == blob
    for k in range(3):
        np.testing.assert_array_equal(m2.coefs(k), m.coefs(k))
    # 4-way data through the d-way compress
    w4 = _workload4()
    p4 = fst.make_params_d(d=4, dtype=fst.FST_F64, lo=w4.lo, hi=w4.hi, grid=(8,) * 4, rank=(3, 3, 2, 2),
                           degree=(6,) * 4, interp_fraction=0.3, n_samples=1000, seed=w4.seed, wavelet=(2, 1))
    m4 = fst.fst_compress_host_d(p4, w4.soa()[:4], w4.soa()[4])
    mo4 = pipeline.compress(w4.pts, w4.vals, w4.lo, w4.hi, (8,) * 4, (3, 3, 2, 2), (6,) * 4, 0.3, w4.seed,
                            wavelet=(2, 1))
    for k in range(4):
        np.testing.assert_array_equal(m4.coefs(k) != 0, mo4.coefs[k] != 0)
        assert rel_l2(m4.coefs(k), mo4.coefs[k]) <= 1e-10


def test_wavelet_parameters_are_validated():
    for wav in [(8, 0), (2, 12), (7, 1), (-1, 0)]:      # level, degree > p, too many details, level
        p = fst.make_params(degree=(9, 9, 9), wavelet=wav)
        assert fst._fn["fst_fit_workspace_bytes"](ctypes.byref(p), 10000) == 0
    core, coefs = datagen.random_model_parts(1, (2, 2, 2), (4, 4, 4))
    with pytest.raises(ValueError):
        fst.fst_model_from_parts((-1.0,) * 3, (1.0,) * 3, (2, 2, 2), (4, 4, 4), core, coefs,
                                 wavelet=((1, 1),) * 3)     # coefficient rows do not match
    big = [np.zeros((5 + 2 * 1, 2)), np.zeros((5 + 2 * 1, 2)), np.zeros((5 + 2 * 511, 2))]
    with pytest.raises(fst.FstError):
        fst.fst_model_from_parts((-1.0,) * 3, (1.0,) * 3, (2, 2, 2), (4, 4, 4), core, big,
                                 wavelet=((1, 1), (1, 1), (9, 1)))


def test_dense_route_sizes_and_argument_checks():
    # workspace of the dense Gram route: the A^T v partials plus R x (M rounded up to 64) rows
    # of the row dtype; 0 for 4-way models, no rows or an unknown dtype.  The argument checks
    # of fst_design_rows / fst_gram_rows fail before any device work.
    core, coefs = datagen.random_model_parts(2, (3, 4, 5), (4, 5, 6))
    m = fst.fst_model_from_parts((0, 0, 0), (1, 1, 1), (3, 4, 5), (4, 5, 6), core, coefs)
    base = fst.fst_gram_workspace_bytes(m, 1000)
    for dt, es in ((fst.FST_F32, 4), (fst.FST_F64, 8)):
        got = fst.fst_gram_dense_workspace_bytes(m, dt, 1000)
        assert got >= base + es * 60 * 1024 and got < base + es * 60 * 1024 + 512
    assert fst.fst_gram_dense_workspace_bytes(m, fst.FST_F32, 0) == 0
    assert fst.fst_gram_dense_workspace_bytes(m, 7, 1000) == 0
    assert fst.fst_gram_dense_workspace_bytes(_model4()[1], fst.FST_F32, 1000) == 0
    fake = ctypes.c_void_p(256)             # never dereferenced: every call below is rejected
    bad_design = [(1000, 1000), (1000, 960), (0, 64)]   # Sp not a multiple of 64; Sp < mrows; no rows
    for mrows, Sp in bad_design:
        st = fst._fn["fst_design_rows"](m.handle, fst.FST_F32, mrows, fake, None, Sp, fake, None, None)
        assert st == fst.FST_E_INVAL, (mrows, Sp)
    st = fst._fn["fst_design_rows"](m.handle, fst.FST_F32, 100, fake, None, 128, fake, fake, None)
    assert st == fst.FST_E_INVAL and "values" in fst.fst_last_error()       # b without vs
    assert fst._fn["fst_design_rows"](None, fst.FST_F32, 100, fake, None, 128, fake, None, None) == fst.FST_E_INVAL
    for R, Sp in ((0, 64), (60, 0), (60, 100)):
        assert fst._fn["fst_gram_rows"](fst.FST_F32, R, Sp, fake, None, fake, None, 0, None) == fst.FST_E_INVAL
    assert fst._fn["fst_gram_rows"](fst.FST_F32, 60, 64, fake, None, None, None, 0, None) == fst.FST_E_INVAL
    assert fst._fn["fst_gram_rows"](fst.FST_F32, 60, 64, fake, None, None, fake, 0, None) == fst.FST_E_INVAL
    assert fst._fn["fst_gram_rows"](fst.FST_F32, 1 << 20, 1 << 21, fake, None, fake, None, 0,
                                    None) == fst.FST_E_UNSUPPORTED


def test_size_queries_need_no_device():
    # every workspace size is a function of the arguments alone (no device query), so it can
    # be taken on a machine without a GPU and gives the same answer on any one
    core, coefs = datagen.random_model_parts(3, (6, 5, 4), (8, 8, 8))
    m = fst.fst_model_from_parts((0, 0, 0), (1, 1, 1), (6, 5, 4), (8, 8, 8), core, coefs)
    g = fst.fst_gram_workspace_bytes(m, 5000)
    assert g >= 8 * 120
    assert fst.fst_refit_workspace_bytes(m, fst.FST_F32, 5000, 0) > g
    assert fst.fst_refit_workspace_bytes(m, fst.FST_F64, 5000, 3) > g
    assert fst.fst_refine_workspace_bytes(m, 5000) > g
    assert fst._fn["fst_residual_workspace_bytes"](m.handle, 5000) > g
    p = fst.make_params(rank=(6, 5, 4), grid=(8, 8, 8), degree=(8, 8, 8), n_samples=5000)
    assert fst.fst_fit_workspace_bytes(p, 100000) > 0
    assert fst._fn["fst_refit_core_mixed_workspace_bytes"](m.handle, fst.FST_F32, 100000, 5000) > 0


def test_model_factor_compressed_columns():
    # the sparse factors of a host compress (Legendre + wavelets) as compressed columns: the
    # same non-zeros as the dense form, rows ascending in every column, counts that add up
    w = datagen.small_f64(n=6000, n_samples=1500)
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=(16, 16, 16), rank=(6, 5, 4), degree=(9, 9, 9),
                        interp_fraction=0.2, n_samples=1500, seed=w.seed, wavelet=(2, 3))
    m = fst.fst_compress_host(p, *w.soa())
    total = 0
    for k in range(3):
        C = m.coefs(k)
        colptr, rowidx, vals = fst.fst_model_factor(m, k)
        assert colptr[0] == 0 and np.all(np.diff(colptr) >= 0) and colptr[-1] == rowidx.size == vals.size
        dense = np.zeros_like(C)
        for j in range(C.shape[1]):
            rows = rowidx[colptr[j]:colptr[j + 1]]
            assert np.all(np.diff(rows) > 0) and np.all((rows >= 0) & (rows < C.shape[0]))
            dense[rows, j] = vals[colptr[j]:colptr[j + 1]]
        np.testing.assert_array_equal(dense, C)
        assert np.count_nonzero(vals) == vals.size == np.count_nonzero(C)
        total += vals.size
    assert total == m.info()["nnz"]
    with pytest.raises(fst.FstError):
        fst.fst_model_factor(m, 3)
