"""Pins of the oracle's mixed least-squares rows (Algorithm 2 steps 2-4, ``oracle.mixing``):
the transform against the explicit Hadamard matrix, its orthogonality and involution, the
sign stream's definition and balance, the exact recovery of the full least-squares solution
when every mixed row is kept (an orthogonal transform leaves the problem unchanged), and the
leverage spreading that motivates the mixing."""
import numpy as np
import pytest
import scipy.linalg

from datagen import random_model_parts
from oracle import mixing
from oracle.lsq import design_rows, factor_values, solve_lstsq
from oracle.model import Model
from oracle.sampler import splitmix64, stream_state


def _model(seed=0, rank=(3, 4, 2), degree=(5, 4, 6)):
    core, coefs = random_model_parts(seed, rank, degree)
    return Model((-1.0,) * 3, (1.0,) * 3, tuple(rank), tuple(degree), core, coefs)


@pytest.mark.parametrize("N", [1, 2, 8, 64, 256])
def test_fwht_is_the_sylvester_hadamard_product(N):
    X = np.random.default_rng(N).standard_normal((N, 3))
    np.testing.assert_allclose(mixing.fwht(X), scipy.linalg.hadamard(N) @ X, atol=1e-12)


def test_fwht_orthogonal_and_involution():
    x = np.random.default_rng(1).standard_normal(1024)
    y = mixing.fwht(x) / np.sqrt(1024)
    assert abs(np.linalg.norm(y) - np.linalg.norm(x)) <= 1e-12 * np.linalg.norm(x)
    np.testing.assert_allclose(mixing.fwht(mixing.fwht(x)), 1024 * x, atol=1e-9)


def test_next_pow2_and_signs():
    assert [mixing.next_pow2(n) for n in (1, 2, 3, 4, 5, 4096, 4097)] == [1, 2, 4, 4, 8, 4096, 8192]
    assert [mixing.mixed_length(n) for n in (1, 4096, 4097, 70000)] == [4096, 4096, 8192, 131072]
    d = mixing.signs(7, 1 << 16)
    assert set(np.unique(d)) == {-1.0, 1.0}
    z = splitmix64(stream_state(7, 5), 5)
    assert [(-1.0 if int(v) >> 63 else 1.0) for v in z] == list(d[:5])
    assert abs(d.mean()) < 0.02            # a fair coin: |mean| ~ 1 / sqrt(65536)


def test_all_rows_kept_recovers_full_least_squares():
    # S = N: the sampled problem is F D [W; 0], F D [u; 0] with F D orthogonal, whose
    # least-squares solution is that of W, u over all n points
    m = _model(seed=4)           # full-rank coefficient matrices (the design has full rank)
    rng = np.random.default_rng(2)
    n = 300
    pts = rng.uniform(-1, 1, (n, 3))
    vals = rng.standard_normal(n)
    N = mixing.mixed_length(n)
    alpha, G, h = mixing.refit_core_mixed(m, pts, vals, N, seed=11)
    W = design_rows(factor_values(m, pts))
    np.testing.assert_allclose(alpha, solve_lstsq(W, vals), rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(G, W.T @ W, atol=1e-10)
    np.testing.assert_allclose(h, W.T @ vals, atol=1e-10)


def test_planted_core_recovered_from_sampled_mixed_rows():
    # values that lie in the model span are reproduced exactly by any S >= R mixed rows
    m = _model(seed=4)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1, 1, (500, 3))
    W = design_rows(factor_values(m, pts))
    alpha0 = rng.standard_normal(W.shape[1])
    alpha, _, _ = mixing.refit_core_mixed(m, pts, W @ alpha0, 120, seed=5)
    np.testing.assert_allclose(alpha, alpha0, rtol=1e-8, atol=1e-9)


def test_mixing_spreads_leverage():
    # a design whose information sits in a few rows: before mixing the largest leverage is
    # 1 (a row no other row can replace); after mixing every row carries about R / N
    n, R = 512, 4
    W = np.zeros((n, R))
    W[:R, :] = np.eye(R)
    W[R:, :] = 1e-3 * np.random.default_rng(4).standard_normal((n - R, R))
    lev = lambda A: np.sum(np.linalg.qr(A)[0] ** 2, axis=1)
    d = mixing.signs(3, n)
    FW = mixing.fwht(d[:, None] * W) / np.sqrt(n)
    assert lev(W).max() > 0.99
    assert lev(FW).max() < 10 * R / n
