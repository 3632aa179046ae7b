"""GPU parity for models whose modes hold the wavelet space W_{s,q} beside P_p (Sec. 4.2,
Algorithm 1; ``oracle.wavelets``): factor values (k_factor_eval with detail rows), the
reconstruction of 3-way and 4-way wavelet models (k_eval_wave), Algorithm 2 on wavelet factors,
the FP64 residual of the refinement path, the grid preview, and an end-to-end fit with the
per-column choice, all through the C ABI against the oracle.

Tolerances (relative L2): FP64 1e-10; FP32 1e-5 (orthonormal bases, values of order 1).
"""
import numpy as np
import pytest

from oracle import lsq, pipeline
from oracle.model import Model as OModel
from oracle.reconstruct import evaluate, evaluate_tensor_grid, rel_l2
from oracle.wavelets import detail_count

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


def _wmodels(seed, rank, degree, wav, lo=None, hi=None, density=0.5):
    d = len(rank)
    lo = lo or (-1.0,) * d
    hi = hi or (1.0,) * d
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(rank)
    coefs = []
    for k in range(d):
        n = degree[k] + 1 + detail_count(*wav[k])
        C = rng.standard_normal((n, rank[k])) * (rng.random((n, rank[k])) < density)
        C[0] += 1.0
        coefs.append(C / np.sqrt(n))
    om = OModel(tuple(lo), tuple(hi), tuple(rank), tuple(degree), core, coefs, wavelet=tuple(wav))
    gm = fst.fst_model_from_parts(lo, hi, rank, degree, core, coefs, wavelet=wav)
    return om, gm


def _pts(seed, n, lo, hi, dtype):
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return (lo + (hi - lo) * rng.random((n, len(lo)))).astype(dtype)


CASES3 = [   # ranks, degrees, per-mode (s, q): mixed Legendre-only and wavelet modes, ragged sizes
    ((5, 7, 3), (9, 12, 6), ((2, 3), (3, 1), (0, 0))),
    ((8, 6, 9), (15, 11, 13), ((3, 2), (1, 5), (4, 1))),
    ((24, 20, 17), (31, 31, 31), ((5, 3), (3, 3), (2, 7))),
]


@pytest.mark.parametrize("rank,degree,wav", CASES3)
def test_factor_values_with_details(dev, rank, degree, wav):
    print(f"wave factor values rank={rank} wav={wav}", flush=True)
    lo, hi = (0.0, -1.0, 2.0), (4.0, 1.0, 3.0)
    om, gm = _wmodels(1, rank, degree, wav, lo, hi)
    for dtype, tol in ((np.float64, 1e-10), (np.float32, 1e-5)):
        pts = _pts(2, 4001, lo, hi, dtype)
        c = [D(pts[:, k], dev) for k in range(3)]
        U, _ = fst.fst_factor_eval(gm, *c)
        ref = lsq.factor_values(om, pts.astype(np.float64))
        Uh = U.cpu().numpy()
        off = 0
        for k in range(3):
            assert rel_l2(Uh[off:off + rank[k]].T, ref[k]) <= tol
            off += rank[k]


@pytest.mark.parametrize("rank,degree,wav", CASES3)
def test_reconstruction_three_way(dev, rank, degree, wav):
    print(f"wave eval rank={rank} wav={wav}", flush=True)
    lo, hi = (0.0, -1.0, 2.0), (4.0, 1.0, 3.0)
    om, gm = _wmodels(3, rank, degree, wav, lo, hi)
    for dtype, tol, n in ((np.float64, 1e-10, 3001), (np.float32, 1e-5, 70001)):
        pts = _pts(4, n, lo, hi, dtype)
        out = fst.fst_eval(gm, *[D(pts[:, k], dev) for k in range(3)])
        assert rel_l2(out.cpu().numpy(), evaluate(om, pts.astype(np.float64))) <= tol
    # points on the box boundary (t = -1, 1) and on cell edges
    edge = np.stack(np.meshgrid(np.linspace(lo[0], hi[0], 9), np.linspace(lo[1], hi[1], 9),
                                np.linspace(lo[2], hi[2], 9), indexing="ij"), -1).reshape(-1, 3)
    out = fst.fst_eval(gm, *[D(edge[:, k], dev) for k in range(3)])
    assert rel_l2(out.cpu().numpy(), evaluate(om, edge)) <= 1e-10


def test_reconstruction_and_refit_four_way(dev):
    rank, degree, wav = (3, 4, 2, 5), (7, 9, 6, 8), ((2, 3), (0, 0), (3, 1), (1, 4))
    lo, hi = (-1.0, 0.0, -2.0, 0.0), (1.0, 1.0, 2.0, 5.0)
    om, gm = _wmodels(5, rank, degree, wav, lo, hi)
    pts = _pts(6, 20000, lo, hi, np.float64)
    c = [D(pts[:, k], dev) for k in range(4)]
    f = fst.fst_eval_d(gm, c)
    assert rel_l2(f.cpu().numpy(), evaluate(om, pts)) <= 1e-10
    vals = evaluate(om, pts) + 0.05 * np.random.default_rng(7).standard_normal(20000)
    alpha_o, _, _, _ = lsq.refit_core(om, pts, vals, 6000, seed=9)
    out = fst.fst_refit_core_d(gm, c, D(vals, dev), 6000, 9)
    assert rel_l2(out.core, alpha_o) <= 1e-10
    assert out.wavelets() == tuple(wav)


def test_refit_and_residual_three_way(dev):
    rank, degree, wav = (6, 5, 7), (11, 9, 13), ((3, 2), (2, 1), (2, 3))
    om, gm = _wmodels(11, rank, degree, wav)
    pts = _pts(12, 30000, (-1.0,) * 3, (1.0,) * 3, np.float64)
    vals = evaluate(om, pts) + 0.05 * np.random.default_rng(13).standard_normal(30000)
    c = [D(pts[:, k], dev) for k in range(3)]
    v = D(vals, dev)
    alpha_o, idx, _, _ = lsq.refit_core(om, pts, vals, 8000, seed=15)
    out = fst.fst_refit_core(gm, *c, v, 8000, 15, gram_prec=fst.FST_GRAM_F64)
    assert rel_l2(out.core.reshape(-1), alpha_o.reshape(-1)) <= 1e-10
    # FP64 normal-equation residual at a trial core (the refinement path's wavelet reconstruction)
    trial = np.random.default_rng(16).standard_normal(int(np.prod(rank)))
    r = fst.fst_residual(gm, *c, v, D(idx.astype(np.int32), dev), D(trial, dev))
    r_ref = lsq.residual_normal(om, pts[idx], vals[idx], trial)
    assert rel_l2(r.cpu().numpy(), r_ref) <= 1e-10


def test_grid_preview_of_wavelet_model(dev):
    rank, degree, wav = (4, 6, 5), (9, 11, 8), ((3, 1), (0, 0), (2, 2))
    lo, hi = (0.0, -1.0, 2.0), (4.0, 1.0, 3.0)
    om, gm = _wmodels(21, rank, degree, wav, lo, hi)
    rng = np.random.default_rng(22)
    gx, gy, gz = rng.uniform(0, 4, 37), rng.uniform(-1, 1, 1), rng.uniform(2, 3, 29)
    out = fst.fst_eval_grid(gm, D(gx, dev), D(gy, dev), D(gz, dev))
    assert rel_l2(out.cpu().numpy(), evaluate_tensor_grid(om, gx, gy, gz)) <= 1e-10


def test_fit_end_to_end_with_wavelet_choice(dev):
    import datagen
    w = datagen.small_f64()
    wav = (3, 2)
    mo = pipeline.fit(w.pts, w.vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction, w.n_samples,
                      w.seed, wavelet=wav)
    p = fst.make_params(dtype=fst.FST_F64, lo=w.lo, hi=w.hi, grid=w.grid, rank=w.rank, degree=w.degree,
                        interp_fraction=w.interp_fraction, n_samples=w.n_samples, seed=w.seed, wavelet=wav)
    c = [D(a, dev) for a in w.soa()]
    gm = fst.fst_fit(p, *c)
    n_wave = 0
    for k in range(3):
        np.testing.assert_array_equal(gm.coefs(k) != 0, mo.coefs[k] != 0)
        assert rel_l2(gm.coefs(k), mo.coefs[k]) <= 1e-10
        n_wave += int(np.any(mo.coefs[k][w.degree[k] + 1:] != 0, axis=0).sum())
    print(f"columns kept in the wavelet space: {n_wave}", flush=True)
    print(f"core rel-L2 {rel_l2(gm.core, mo.core):.3e}", flush=True)
    assert rel_l2(gm.core, mo.core) <= 1e-10
    f = fst.fst_eval(gm, *c[:3]).cpu().numpy()
    assert abs(rel_l2(f, w.vals) - rel_l2(evaluate(mo, w.pts), w.vals)) <= 1e-8
