"""GPU parity of Algorithm 2 with its randomised mixing (fst_refit_core_mixed: sign flips,
normalised Walsh-Hadamard transform over N = max(4096, 2^ceil(log2 n)) rows, uniform
sampling of S rows, FP64 Cholesky) through the C ABI, against the oracle's mixed problem
(``oracle.mixing``, pinned on the CPU) and against the unmixed full least-squares solution
when every mixed row is kept.

Tolerances (relative L2 of the core): FP64 1e-10; FP32 1e-5 on a well-conditioned design
(orthonormal factor functions, uniform points: kappa(G) of order 1, so FP32 rows and
transform rounding stay near 1e-6).
"""
import numpy as np
import pytest

from oracle import mixing
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


def _models(seed, rank, degree, orthonormal=False):
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(tuple(rank))
    if orthonormal:
        coefs = [np.linalg.qr(rng.standard_normal((degree[k] + 1, rank[k])))[0] for k in range(3)]
    else:
        coefs = [rng.standard_normal((degree[k] + 1, rank[k])) / np.sqrt(degree[k] + 1) for k in range(3)]
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    return (OModel(lo, hi, tuple(rank), tuple(degree), core, coefs),
            fst.fst_model_from_parts(lo, hi, rank, degree, core, coefs))


def _data(seed, n, om, dtype):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, (n, 3)).astype(dtype)
    # a field near the model span plus noise (the sampled problem is not consistent)
    from oracle.reconstruct import evaluate
    vals = (evaluate(om, pts.astype(np.float64)) + 0.1 * rng.standard_normal(n)).astype(dtype)
    return pts, vals


# n = 3000: N = 4096 (one block, second pass only scatters); n = 40000: N = 65536, four
# cross-block stages (register passes of three and one); n = 70000: N = 131072, five (three and
# two); ranks not multiples of 8
@pytest.mark.parametrize("n,rank,degree,S", [
    (3000, (4, 5, 3), (7, 7, 7), 1500),
    (40000, (5, 4, 6), (8, 7, 9), 2500),
    (70000, (6, 5, 4), (9, 8, 7), 3000),
])
def test_mixed_refit_fp64_matches_oracle(dev, n, rank, degree, S):
    print(f"mixed fp64 n={n} rank={rank} S={S}", flush=True)
    om, gm = _models(n, rank, degree)
    pts, vals = _data(1, n, om, np.float64)
    seed = 17
    alpha_o, _, _ = mixing.refit_core_mixed(om, pts, vals, S, seed)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    out = fst.fst_refit_core_mixed(gm, x, y, z, D(vals, dev), S, seed)
    assert rel_l2(out.core.reshape(-1), alpha_o) <= 1e-10


def test_mixed_refit_fp32_matches_oracle(dev):
    n, rank, degree, S = 70000, (8, 6, 5), (11, 9, 8), 4000
    print(f"mixed fp32 n={n} rank={rank} S={S}", flush=True)
    om, gm = _models(5, rank, degree, orthonormal=True)
    pts, vals = _data(2, n, om, np.float32)
    seed = 23
    alpha_o, _, _ = mixing.refit_core_mixed(om, pts.astype(np.float64), vals.astype(np.float64), S, seed)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    out = fst.fst_refit_core_mixed(gm, x, y, z, D(vals, dev), S, seed)
    assert rel_l2(out.core.reshape(-1), alpha_o) <= 1e-5


def test_all_mixed_rows_give_the_full_least_squares_core(dev):
    # S = N: F D is orthogonal, so the mixed problem over all N rows has the solution of the
    # unmixed problem over all n points (the plain refit with n_samples = n)
    n, rank, degree = 5000, (5, 4, 6), (8, 8, 8)
    print(f"mixed all rows n={n}", flush=True)
    om, gm = _models(9, rank, degree)
    pts, vals = _data(3, n, om, np.float64)
    x, y, z, v = [D(pts[:, k], dev) for k in range(3)] + [D(vals, dev)]
    N = mixing.mixed_length(n)
    mixed = fst.fst_refit_core_mixed(gm, x, y, z, v, N, 4)
    full = fst.fst_refit_core(gm, x, y, z, v, n, 4)
    assert rel_l2(mixed.core, full.core) <= 1e-10


def test_mixed_refit_rejects_bad_sample_counts(dev):
    om, gm = _models(2, (3, 3, 3), (5, 5, 5))
    pts, vals = _data(4, 500, om, np.float64)
    x, y, z, v = [D(pts[:, k], dev) for k in range(3)] + [D(vals, dev)]
    for S in (27, 4097):
        with pytest.raises(fst.FstError) as e:
            fst.fst_refit_core_mixed(gm, x, y, z, v, S, 1)
        assert e.value.status == fst.FST_E_INVAL
