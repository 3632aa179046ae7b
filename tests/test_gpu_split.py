"""Split 16-bit Gram of the precision form (eq. (6) on 16-bit MFMA): design rows split into two
FP16 terms (scaled), three BF16 terms or two BF16 terms; G = the sum of the kept term products,
FP32 sums folded into FP64.  Parity against the FP64 oracle at the FP32 bar (1e-5) on
sizes that span several 128 x 128 tiles and tile groups, ragged row and column counts, and
the refit with three FP64-residual refinement steps against the oracle's core at 1e-6."""
import numpy as np
import pytest

import datagen
from oracle import lsq, pipeline
from oracle.model import Model as OModel
from oracle.reconstruct import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
fst = pytest.importorskip("paper_1907_05884_amd.binding")

SPLITS = [("f16x2", 4), ("bf16x3", 5), ("bf16x2", 6)]
# unit roundoff of the split representation of an entry: 2 x 11 bits (FP16), 3 x 8 (BF16 x 3),
# 2 x 8 (BF16 x 2)
UNIT = {4: 2.0 ** -22, 5: 2.0 ** -24, 6: 2.0 ** -16}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def D(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def H(t):
    return t.detach().cpu().numpy()


def _case(seed, rank, degree, m):
    core, coefs = datagen.random_model_parts(seed, rank, degree)
    om = OModel((-1,) * 3, (1,) * 3, tuple(rank), tuple(degree), core, coefs)
    gm = fst.fst_model_from_parts((-1,) * 3, (1,) * 3, rank, degree, core, coefs)
    pts = np.random.default_rng(seed + 1).uniform(-1, 1, (m, 3)).astype(np.float32)
    return om, gm, pts


def test_split_constants():
    assert (fst.FST_GRAM_F16X2, fst.FST_GRAM_BF16X3, fst.FST_GRAM_BF16X2) == (4, 5, 6)


# R = 504 (4 tiles, ragged), 1331 (11 tiles: tile groups beyond the first column group),
# 8 (one partial tile); M ragged against the 64-row chunks, M < 64, M a multiple of 64
@pytest.mark.parametrize("name,code", SPLITS)
@pytest.mark.parametrize("rank,degree,m", [((9, 8, 7), (15, 15, 15), 6007), ((11, 11, 11), (20, 20, 20), 3001),
                                           ((2, 2, 2), (3, 3, 3), 50), ((5, 7, 3), (9, 12, 6), 1344)])
def test_split_gram_parity(dev, name, code, rank, degree, m):
    om, gm, pts = _case(40, rank, degree, m)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    G, _ = fst.fst_gram(gm, U, gram_prec=code)
    A = lsq.design_rows(lsq.factor_values(om, pts.astype(np.float64)))
    Gr = A.T @ A
    bound = np.abs(A).T @ np.abs(A)
    low = np.tril_indices(om.R)
    Gh = H(G)
    # every entry within max(1e-5, 4u) of sum_q |A_qi A_qj| of the FP64 value, and the lower
    # triangle within that in relative L2: the FP32 bar for FP16 x 2 and BF16 x 3 (a single
    # 16-bit term would miss it by 100x)
    tol = max(1e-5, 4 * UNIT[code])
    assert np.all(np.abs(Gh[low] - Gr[low]) <= tol * bound[low])
    assert rel_l2(Gh[low], Gr[low]) <= tol
    # against the library's FP32 Gram of the same factor values
    G32, _ = fst.fst_gram(gm, U)
    assert rel_l2(Gh[low], H(G32)[low]) <= max(2e-6, 4 * UNIT[code])
    # deterministic, strictly upper part untouched
    G2, _ = fst.fst_gram(gm, U, gram_prec=code)
    assert torch.equal(G, G2)
    assert np.all(Gh[np.triu_indices(om.R, 1)] == 0.0)


@pytest.mark.parametrize("name,code", SPLITS)
def test_split_gram_needs_its_workspace(dev, name, code):
    _, gm, pts = _case(41, (6, 5, 4), (9, 9, 9), 700)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    U, _ = fst.fst_factor_eval(gm, x, y, z)
    need = fst.fst_gram_split_workspace_bytes(gm, code, 700)
    assert need > fst.fst_gram_workspace_bytes(gm, 700)
    assert fst.fst_gram_split_workspace_bytes(gm, fst.FST_GRAM_F32, 700) == 0
    ws = torch.empty(need - 4096, dtype=torch.uint8, device=dev)
    with pytest.raises(fst.FstError) as e:
        fst.fst_gram(gm, U, gram_prec=code, ws=ws)
    assert e.value.status == fst.FST_E_NOMEM


@pytest.mark.parametrize("name,code", SPLITS)
def test_refit_split_gram_three_steps_matches_fp64(dev, name, code):
    w = datagen.small_f64()
    m0 = pipeline.compress(w.pts, w.vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction, w.seed)
    wl = datagen.make_workload("lp", seed=3, n=40000, n_gauss=6, grid=(32, 32, 32), rank=(8, 8, 8),
                               degree=(15, 15, 15), interp_fraction=0.1, n_samples=4000, dtype=np.float32)
    alpha_o, _, _, _ = lsq.refit_core(m0, wl.pts.astype(np.float64), wl.vals.astype(np.float64), 4000, 9)
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, m0.core, m0.coefs)
    x, y, z, v = [D(a, dev) for a in wl.soa()]
    errs = []
    for steps in (0, 3):
        out = fst.fst_refit_core(gm, x, y, z, v, 4000, 9, gram_prec=code, refine_steps=steps)
        info = out.solve_info()
        assert info["gram_prec"] == code and info["dropped"] == 0, info
        errs.append(rel_l2(out.core, alpha_o))
    assert errs[0] <= 1e-4, errs
    assert errs[1] <= 1e-6, errs


@pytest.mark.parametrize("name,code", SPLITS)
def test_tile_order_autotuner(dev, name, code, tmp_path, monkeypatch):
    # the split Gram's tile-group shape is picked per shape by timing the candidates on the first
    # call; with FST_TUNE_FILE the choice is kept in that JSON object.  Every candidate must give
    # the same G bit for bit: forcing each one through the file checks it.
    import json
    om, gm, pts = _case(41, (9, 10, 7), (11, 11, 11), 5000)    # R = 630: 5 x 5 tiles
    U, _ = fst.fst_factor_eval(gm, *[D(pts[:, k], dev) for k in range(3)])
    path = tmp_path / "tune.json"
    monkeypatch.setenv("FST_TUNE_FILE", str(path))
    G1, _ = fst.fst_gram(gm, U, gram_prec=code)        # tunes and records
    G2, _ = fst.fst_gram(gm, U, gram_prec=code)        # takes the recorded choice
    torch.cuda.synchronize()
    tab = json.loads(path.read_text())
    keys = [k for k in tab if k.startswith(f"split:{code}:nt5:")]
    assert len(keys) == 1 and tab[keys[0]] in (0, 1, 2), tab
    assert torch.equal(torch.tril(G1), torch.tril(G2))
    for choice in (0, 1, 2):
        tab[keys[0]] = choice
        path.write_text(json.dumps(tab))
        monkeypatch.setenv("FST_TUNE_FILE", str(tmp_path / "other.json"))
        fst.fst_gram(gm, U, gram_prec=code)            # a call under another file ...
        monkeypatch.setenv("FST_TUNE_FILE", str(path))
        Gc, _ = fst.fst_gram(gm, U, gram_prec=code)    # ... makes this one reload the edited file
        torch.cuda.synchronize()
        assert torch.equal(torch.tril(Gc), torch.tril(G1)), choice
