"""GPU parity of fst_solve_core (Algorithm 2 step 5 from the caller's normal equations: FP64
Cholesky, solve, FP64-residual refinement with the precision ladder) through the C ABI:

* FP64 rows and Gram on the 20,000-point workload's model (M = 2,000): the core equals the
  oracle's FP64 core of the same sample to 1e-10 without refinement and with two steps, and
  equals fst_refit_core's core (the same calls after the same Gram) to 1e-13;
* FP32 points with a split BF16 x 2 Gram and three refinement steps: the refinement reaches a
  relative normal-equation residual of 1e-8 or below and the core is within 1e-6 of the
  oracle's FP64 core (the design is well conditioned, kappa(G) of order 1e3);
* a workspace below fst_solve_core_workspace_bytes is refused with FST_E_NOMEM, and so is a
  split Gram without room for its copy.
"""
import numpy as np
import pytest

import datagen
from oracle import lsq, pipeline
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


@pytest.fixture(scope="module")
def small():
    w = datagen.small_f64()
    m0 = pipeline.compress(w.pts, w.vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction, w.seed)
    return w, m0


def _system(gm, w, dev, dtype, gram_prec):
    pts, vals = w.pts.astype(dtype), w.vals.astype(dtype)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    v = D(vals, dev)
    idx = D(fst.fst_sample_indices(w.seed, fst.FST_STREAM_LS, w.n, w.n_samples).astype(np.int32), dev)
    U, vs = fst.fst_factor_eval(gm, x, y, z, v, idx)
    G, h = fst.fst_gram(gm, U, vs, gram_prec=gram_prec)
    return x, y, z, v, idx, U, vs, G, h


@pytest.mark.parametrize("steps", [0, 2])
def test_solve_core_fp64_matches_oracle_and_refit(dev, small, steps):
    w, m0 = small
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, m0.core, m0.coefs)
    alpha_o, *_ = lsq.refit_core(m0, w.pts, w.vals, w.n_samples, w.seed)
    x, y, z, v, idx, U, vs, G, h = _system(gm, w, dev, np.float64, fst.FST_GRAM_F64)
    alpha, info = fst.fst_solve_core(gm, x, y, z, v, idx, U, vs, G, h, refine_steps=steps)
    a = alpha.cpu().numpy()
    assert info["gram_prec"] == fst.FST_GRAM_F64 and info["dropped"] == 0
    assert rel_l2(a, alpha_o.reshape(-1)) <= 1e-10
    ref = fst.fst_refit_core(gm, x, y, z, v, w.n_samples, w.seed, refine_steps=steps)
    assert rel_l2(a, ref.core.reshape(-1)) <= 1e-13
    if steps:
        assert info["rel_residual"] <= 1e-12


def test_solve_core_split_gram_refines_to_oracle(dev, small):
    w, m0 = small
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, m0.core, m0.coefs)
    x, y, z, v, idx, U, vs, G, h = _system(gm, w, dev, np.float32, fst.FST_GRAM_BF16X2)
    alpha, info = fst.fst_solve_core(gm, x, y, z, v, idx, U, vs, G, h, gram_prec=fst.FST_GRAM_BF16X2,
                                     refine_steps=3)
    print("split solve info", info, flush=True)
    assert info["gram_prec"] in (fst.FST_GRAM_BF16X2, fst.FST_GRAM_F64) and info["rel_residual"] <= 1e-8
    alpha_o, *_ = lsq.refit_core(m0, w.pts.astype(np.float32).astype(np.float64),
                                 w.vals.astype(np.float32).astype(np.float64), w.n_samples, w.seed)
    assert rel_l2(alpha.cpu().numpy(), alpha_o.reshape(-1)) <= 1e-6


def test_solve_core_rejects_small_workspace(dev, small):
    w, m0 = small
    gm = fst.fst_model_from_parts(w.lo, w.hi, w.rank, w.degree, m0.core, m0.coefs)
    x, y, z, v, idx, U, vs, G, h = _system(gm, w, dev, np.float32, fst.FST_GRAM_BF16X2)
    need = int(fst._fn["fst_solve_core_workspace_bytes"](gm.handle, w.n_samples, fst.FST_GRAM_BF16X2))
    plain = int(fst._fn["fst_solve_core_workspace_bytes"](gm.handle, w.n_samples, fst.FST_GRAM_F32))
    assert need >= plain + 8 * gm.R * gm.R
    for nbytes in (plain // 2, need - 256):
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        with pytest.raises(fst.FstError) as e:
            fst.fst_solve_core(gm, x, y, z, v, idx, U, vs, G, h, gram_prec=fst.FST_GRAM_BF16X2, ws=ws)
        assert e.value.status == fst.FST_E_NOMEM
