"""GPU tests of the batched form through the C ABI.

The batched fit runs Algorithm 1 per variable on host threads (one shared interpolation
subset), forms the Gram matrices of all variables in one persistent launch and solves each
variable in FP64.  Its results must equal the per-variable entry points on the same inputs
(the same kernels do the same arithmetic, so the bound is a few units of rounding), and the
FP64 form must match the oracle to 1e-10.  The batched reconstruction and its captured graph
must equal per-variable reconstruction exactly, on every replay.
"""
import numpy as np
import pytest

import datagen
from oracle import lsq, reconstruct
from oracle.model import Model as OModel
from oracle.reconstruct import rel_l2

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


def _omodel(wl, m):
    inf = m.info()
    return OModel(tuple(wl.lo), tuple(wl.hi), tuple(inf["rank"]), tuple(inf["degree"]),
                  m.core.reshape(inf["rank"]), [m.coefs(k) for k in range(3)])


def _params(wl, dtype, rank, degree, gram_prec, refine=0):
    return fst.make_params(dtype=dtype, lo=wl.lo, hi=wl.hi, grid=wl.grid, rank=rank,
                           degree=(degree,) * 3, interp_fraction=wl.interp_fraction,
                           n_samples=wl.n_samples, seed=wl.seed, gram_prec=gram_prec,
                           refine_steps=refine)


class Case:
    def __init__(self, wl, dev, np_dtype):
        self.wl = wl
        self.np_dtype = np_dtype
        self.pts = wl.pts.astype(np_dtype)
        self.vals = [v.astype(np_dtype) for v in wl.vals]
        self.xyz = [D(np.ascontiguousarray(self.pts[:, k]), dev) for k in range(3)]
        self.dv = [D(v, dev) for v in self.vals]


def _fit_both(case, dtype, gram_prec, refine):
    """Batched fit, and the same problems through the per-variable entry points."""
    wl = case.wl
    base = _params(wl, dtype, wl.ranks[0], wl.degrees[0], gram_prec, refine)
    models, t, used = fst.fst_fit_batched(base, wl.ranks, wl.degrees, *case.xyz, case.dv)
    assert len(models) == len(wl.vals) and np.all(t >= 0)
    assert np.all(used == gram_prec)
    refs = []
    for v, (r, p) in enumerate(zip(wl.ranks, wl.degrees)):
        pv = _params(wl, dtype, r, p, gram_prec, refine)
        cols = [np.ascontiguousarray(case.pts[:, k]) for k in range(3)]
        host = fst.fst_compress_host(pv, *cols, case.vals[v])
        refs.append((host, fst.fst_refit_core(host, *case.xyz, case.dv[v], wl.n_samples, wl.seed + v,
                                              gram_prec=gram_prec, refine_steps=refine)))
    return models, refs


@pytest.fixture(scope="module")
def small64(dev):
    wl = datagen.batched(n_vars=5, n=60_000, grid=(24, 24, 24), rmin=3, rmax=9, pmin=9, pmax=15)
    case = Case(wl, dev, np.float64)
    models, refs = _fit_both(case, fst.FST_F64, fst.FST_GRAM_F64, 0)
    return case, models, refs


def test_batched_fit_f64_matches_per_variable(small64):
    case, models, refs = small64
    for v, (m, (host, ref)) in enumerate(zip(models, refs)):
        assert m.rank == tuple(case.wl.ranks[v])
        for k in range(3):
            np.testing.assert_allclose(m.coefs(k), host.coefs(k), rtol=0, atol=1e-13)
        assert rel_l2(m.core, ref.core) <= 1e-12, v


def test_batched_fit_f64_matches_oracle(small64):
    """Variable v refits with seed + v: the oracle's Algorithm 2 on the same model."""
    case, models, _ = small64
    for v in (0, 3):
        om = _omodel(case.wl, models[v])
        alpha, *_ = lsq.refit_core(om, case.pts, case.vals[v], case.wl.n_samples, case.wl.seed + v)
        assert rel_l2(models[v].core.reshape(-1), alpha.reshape(-1)) <= 1e-10, v


def test_batched_eval_and_graph_replays(small64, dev):
    case, models, _ = small64
    x, y, z = case.xyz
    eager = [fst.fst_eval(m, x, y, z) for m in models]
    outs = fst.fst_eval_batched(models, x, y, z)
    for a, b in zip(outs, eager):
        assert torch.equal(a, b)
    # against the oracle at sampled points
    idx = np.random.default_rng(0).choice(case.pts.shape[0], 2000, replace=False)
    for v in (1, 4):
        ref = reconstruct.evaluate(_omodel(case.wl, models[v]), case.pts[idx])
        assert rel_l2(eager[v].cpu().numpy()[idx], ref) <= 1e-10
    gouts = [torch.empty_like(x) for _ in models]
    g = fst.EvalGraph(models, x, y, z, gouts)
    scratch = torch.empty_like(x)
    for rep in range(4):
        for o in gouts:
            o.fill_(float("nan"))
        fst.fst_eval(models[rep % len(models)], x, y, z, out=scratch)      # eager work between replays
        g.launch()
        torch.cuda.synchronize()
        for a, b in zip(gouts, eager):
            assert torch.equal(a, b), rep
    fst.fst_graph_free(g)
    fst.fst_graph_free(g)   # second free is a no-op


def test_batched_fit_f32_low_precision_matches_per_variable(dev):
    """FP32 data, BF16 and FP16 Gram, FP64-residual refinement: same arithmetic as the
    per-variable path; refinement drives the core toward the FP64 solution of the same rows."""
    wl = datagen.batched(n_vars=4, n=80_000, grid=(24, 24, 24), rmin=4, rmax=8, pmin=11, pmax=15)
    case = Case(wl, dev, np.float32)
    for prec in (fst.FST_GRAM_BF16, fst.FST_GRAM_F16):
        models, refs = _fit_both(case, fst.FST_F32, prec, 4)
        for v, (m, (host, ref)) in enumerate(zip(models, refs)):
            assert rel_l2(m.core, ref.core) <= 1e-12, (prec, v)
        om = _omodel(wl, models[1])
        alpha, _, Gk, _ = lsq.refit_core(om, case.pts.astype(np.float64), case.vals[1], wl.n_samples, wl.seed + 1)
        err = rel_l2(models[1].core.reshape(-1), alpha.reshape(-1))
        info = models[1].solve_info()
        kappa = np.linalg.cond(Gk)
        print(f"prec {prec}: core rel-L2 vs FP64 oracle after refinement {err:.3e} ({info}, kappa {kappa:.2e})")
        # the refinement stops at a relative normal-equation residual of 1e-8 or below (after at most
        # four times the steps asked for, climbing to a wider Gram if needed): the core is then within
        # kappa(G) times that residual, plus the FP32 rounding of the points and values
        assert info["rel_residual"] <= 1e-8
        assert err <= max(1e-6, 2 * kappa * info["rel_residual"])


def test_batched_more_variables_than_one_launch(dev):
    """More variables than one persistent launch holds: the Gram work is split."""
    wl = datagen.batched(n_vars=50, n=20_000, grid=(16, 16, 16), rmin=3, rmax=5, pmin=9, pmax=13)
    case = Case(wl, dev, np.float64)
    models, refs = _fit_both(case, fst.FST_F64, fst.FST_GRAM_F64, 0)
    for v, (m, (_, ref)) in enumerate(zip(models, refs)):
        assert rel_l2(m.core, ref.core) <= 1e-12, v


def test_batched_rank_deficient_variable(dev):
    """At degree 6 on a 12^3 grid the sparse fits of variable 7 give collinear factor
    functions (the oracle's sampled Gram has smallest eigenvalue ~1e-16 of the largest), so
    its least-squares problem has many solutions.  The FP64 step must skip the dependent
    columns, agree with the per-variable path, and give the field of the minimum-norm
    least-squares solution at the sampled rows."""
    wl = datagen.batched(n_vars=8, n=20_000, grid=(12, 12, 12), rmin=3, rmax=5, pmin=5, pmax=7)
    case = Case(wl, dev, np.float64)
    base = _params(wl, fst.FST_F64, wl.ranks[0], wl.degrees[0], fst.FST_GRAM_F64)
    models, _, used = fst.fst_fit_batched(base, wl.ranks, wl.degrees, *case.xyz, case.dv)
    assert np.all(used == fst.FST_GRAM_F64)
    prec, dropped = models[7].fit_info()
    assert dropped > 0
    assert all(models[v].fit_info()[1] == 0 for v in range(7))
    pv = _params(wl, fst.FST_F64, wl.ranks[7], wl.degrees[7], fst.FST_GRAM_F64)
    host = fst.fst_compress_host(pv, *[np.ascontiguousarray(case.pts[:, k]) for k in range(3)], case.vals[7])
    ref = fst.fst_refit_core(host, *case.xyz, case.dv[7], wl.n_samples, wl.seed + 7)
    assert ref.fit_info() == (fst.FST_GRAM_F64, dropped)
    assert rel_l2(models[7].core, ref.core) <= 1e-12
    # the kept columns carry the least-squares solution restricted to them; skipped columns
    # are within sqrt(2^-26) of the span of the kept ones, so the field differs from the
    # minimum-norm least-squares field by about that much at most
    om = _omodel(wl, models[7])
    idx = lsq.sample_rows(wl.seed + 7, case.pts.shape[0], wl.n_samples)
    A = lsq.design_rows(lsq.factor_values(om, case.pts[idx]))
    core = models[7].core.reshape(-1)
    kept = core != 0
    assert np.count_nonzero(~kept) == dropped
    a_kept = lsq.solve_lstsq(A[:, kept], case.vals[7][idx])
    assert rel_l2(core[kept], a_kept) <= 1e-7
    f_min_norm = A @ lsq.solve_lstsq(A, case.vals[7][idx])
    assert rel_l2(A @ core, f_min_norm) <= 1e-5


def test_batched_errors(small64, dev):
    case, models, _ = small64
    wl = case.wl
    base = _params(wl, fst.FST_F64, wl.ranks[0], wl.degrees[0], fst.FST_GRAM_F64)
    ranks = [list(r) for r in wl.ranks[:2]]
    ranks[1] = [9, 2, 2]            # r1 > r2 r3: not a valid Tucker rank
    with pytest.raises(fst.FstError, match="variable 1"):
        fst.fst_fit_batched(base, ranks, wl.degrees[:2], *case.xyz, case.dv[:2])
    x, y, z = case.xyz
    with pytest.raises(fst.FstError):
        fst.EvalGraph(models, x[:0], y[:0], z[:0], [torch.empty(0, dtype=x.dtype, device=dev)] * len(models))


def test_batched_split_gram_three_steps_matches_oracle(dev):
    """The batched precision form: BF16 x 2 split Grams of all variables (row planes written,
    then one launch over every variable's tiles), concurrent FP64 Cholesky solves and three
    FP64-residual refinement steps.  Every variable's core matches the oracle's FP64 core of
    its own sampled problem to 1e-6, the smallest and the largest R included, and equals the
    per-variable entry point (the same tile arithmetic)."""
    wl = datagen.batched(n_vars=6, n=120_000, grid=(24, 24, 24), rmin=4, rmax=12, pmin=11, pmax=19)
    case = Case(wl, dev, np.float32)
    code = fst.FST_GRAM_BF16X2
    base = _params(wl, fst.FST_F32, wl.ranks[0], wl.degrees[0], code, 3)
    models, t, used = fst.fst_fit_batched(base, wl.ranks, wl.degrees, *case.xyz, case.dv)
    assert np.all(used == code), used
    Rs = [int(np.prod(r)) for r in wl.ranks]
    print("R per variable", Rs)
    for v in range(len(models)):
        om = _omodel(wl, models[v])
        alpha, *_ = lsq.refit_core(om, case.pts.astype(np.float64), case.vals[v].astype(np.float64),
                                   wl.n_samples, wl.seed + v)
        err = rel_l2(models[v].core.reshape(-1), alpha.reshape(-1))
        print(f"variable {v} R={Rs[v]}: core rel-L2 {err:.3e}, fit {models[v].solve_info()}")
        assert err <= 1e-6, (v, Rs[v], err)
    for v in (int(np.argmin(Rs)), int(np.argmax(Rs))):
        pv = _params(wl, fst.FST_F32, wl.ranks[v], wl.degrees[v], code, 3)
        host = fst.fst_compress_host(pv, *[np.ascontiguousarray(case.pts[:, k]) for k in range(3)], case.vals[v])
        ref = fst.fst_refit_core(host, *case.xyz, case.dv[v], wl.n_samples, wl.seed + v, gram_prec=code,
                                 refine_steps=3)
        assert rel_l2(models[v].core, ref.core) <= 1e-12, v


def test_batched_split_gram_tile_orders_agree(dev, tmp_path, monkeypatch):
    """The batched split Gram's tile order (triangle order, 4 x 8 or 8 x 4 groups) is picked by
    timing on first use and kept in the JSON file FST_TUNE_FILE names; forcing each order through
    that file gives the same cores (the Grams agree bit for bit)."""
    import json
    wl = datagen.batched(n_vars=4, n=60_000, grid=(16, 16, 16), rmin=4, rmax=12, pmin=11, pmax=19)
    case = Case(wl, dev, np.float32)
    code = fst.FST_GRAM_BF16X2
    base = _params(wl, fst.FST_F32, wl.ranks[0], wl.degrees[0], code, 3)
    path = tmp_path / "tune.json"
    monkeypatch.setenv("FST_TUNE_FILE", str(path))
    first, *_ = fst.fst_fit_batched(base, wl.ranks, wl.degrees, *case.xyz, case.dv)
    tab = json.loads(path.read_text())
    keys = [k for k in tab if k.startswith(f"split_batched:{code}:")]
    assert keys and all(tab[k] in (0, 1, 2) for k in keys), tab
    for choice in (0, 1, 2):
        for k in keys:
            tab[k] = choice
        path.write_text(json.dumps(tab))
        monkeypatch.setenv("FST_TUNE_FILE", str(tmp_path / "other.json"))
        fst.fst_fit_batched(base, wl.ranks[:1], wl.degrees[:1], *case.xyz, case.dv[:1])   # another file ...
        monkeypatch.setenv("FST_TUNE_FILE", str(path))                                    # ... then reload
        models, *_ = fst.fst_fit_batched(base, wl.ranks, wl.degrees, *case.xyz, case.dv)
        for v in range(len(models)):
            assert rel_l2(models[v].core, first[v].core) <= 1e-12, (choice, v)
