"""Pins of the oracle's least-squares core refit (eq. (6), Algorithm 2) and of the model
evaluation (eq. (1)): brute force on tiny inputs, the Kronecker closed form of the Gram on a
full tensor grid, exact recovery of a planted core, and two independent evaluation forms."""
import numpy as np
import pytest

from datagen import random_model_parts
from oracle.basis import legendre_orthonormal, to_reference
from oracle.interp import grid_nodes, grid_points
from oracle.lsq import (design_rows, factor_values, normal_equations, refit_core,
                        residual_normal, sample_rows, solve_cholesky, solve_lstsq)
from oracle.model import Model, to_csc
from oracle.reconstruct import (evaluate, evaluate_full_expansion, evaluate_on_grid,
                                evaluate_tensor_grid, full_expansion_coefficients, rel_l2)
from oracle.sthosvd import tucker_full


def _model(seed=0, rank=(3, 4, 2), degree=(5, 4, 6), lo=(-1, -1, -1), hi=(1, 1, 1)):
    core, coefs = random_model_parts(seed, rank, degree)
    return Model(tuple(lo), tuple(hi), tuple(rank), tuple(degree), core, coefs)


def _pts(seed, n, lo=(-1, -1, -1), hi=(1, 1, 1)):
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return lo + (hi - lo) * rng.random((n, 3))


def test_factor_values_bruteforce():
    m = _model(lo=(0, 0, 0), hi=(4, 1, 1))
    pts = _pts(1, 7, (0, 0, 0), (4, 1, 1))
    U = factor_values(m, pts)
    for k in range(3):
        for q in range(7):
            xi = 2 * (pts[q, k] - m.lo[k]) / (m.hi[k] - m.lo[k]) - 1
            for j in range(m.rank[k]):
                s = 0.0
                for i in range(m.degree[k] + 1):
                    # classical Legendre by explicit recurrence, scaled to unit norm
                    P = [1.0, xi]
                    for t in range(1, i):
                        P.append(((2 * t + 1) * xi * P[t] - t * P[t - 1]) / (t + 1))
                    s += m.coefs[k][i, j] * np.sqrt(2 * i + 1) * P[i]
                assert U[k][q, j] == pytest.approx(s, rel=1e-12, abs=1e-14)


def test_design_rows_bruteforce_and_kron():
    m = _model()
    pts = _pts(2, 5)
    U1, U2, U3 = factor_values(m, pts)
    A = design_rows((U1, U2, U3))
    r1, r2, r3 = m.rank
    for q in range(5):
        for j1 in range(r1):
            for j2 in range(r2):
                for j3 in range(r3):
                    assert A[q, (j1 * r2 + j2) * r3 + j3] == pytest.approx(
                        U1[q, j1] * U2[q, j2] * U3[q, j3], rel=1e-15)
        np.testing.assert_allclose(A[q], np.kron(np.kron(U1[q], U2[q]), U3[q]), rtol=1e-15)


def test_gram_bruteforce_and_chunking():
    m = _model()
    pts = _pts(3, 50)
    v = np.random.default_rng(3).standard_normal(50)
    G, h = normal_equations(m, pts, v, chunk=7)
    A = design_rows(factor_values(m, pts))
    Gb = np.zeros((m.R, m.R))
    for q in range(50):
        Gb += np.outer(A[q], A[q])
    np.testing.assert_allclose(G, Gb, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(h, A.T @ v, rtol=1e-12, atol=1e-12)


def test_gram_kronecker_closed_form_on_tensor_grid():
    m = _model(rank=(3, 2, 4), degree=(6, 5, 7))
    pts = grid_points((5, 4, 6))     # a full tensor grid of sample points
    G, _ = normal_equations(m, pts, np.zeros(pts.shape[0]), chunk=33)
    Uk = [legendre_orthonormal(grid_nodes(I), m.degree[k]) @ m.coefs[k]
          for k, I in enumerate((5, 4, 6))]
    Gk = [U.T @ U for U in Uk]
    np.testing.assert_allclose(G, np.kron(np.kron(Gk[0], Gk[1]), Gk[2]), rtol=1e-12, atol=1e-12)


def test_exact_recovery_of_planted_core():
    m = _model(rank=(3, 3, 3), degree=(7, 7, 7))
    pts = _pts(4, 3000)
    v = evaluate(m, pts)
    alpha, idx, G, h = refit_core(m, pts, v, 400, seed=11)
    np.testing.assert_allclose(alpha, m.core, rtol=1e-10, atol=1e-10)
    assert len(idx) == 400


def test_full_sample_equals_full_least_squares_and_qr():
    m = _model(rank=(2, 3, 2), degree=(4, 4, 4))
    pts = _pts(5, 300)
    v = np.random.default_rng(5).standard_normal(300)
    alpha, idx, G, h = refit_core(m, pts, v, 300, seed=3)
    np.testing.assert_array_equal(idx, np.arange(300))
    A = design_rows(factor_values(m, pts))
    a_qr = solve_lstsq(A, v)
    kappa = np.linalg.cond(A)
    assert rel_l2(alpha.reshape(-1), a_qr) <= 100 * kappa ** 2 * 2.0 ** -53


def test_row_sign_flips_do_not_change_solution():
    m = _model(rank=(2, 2, 3), degree=(5, 5, 5))
    pts = _pts(6, 200)
    v = np.random.default_rng(6).standard_normal(200)
    A = design_rows(factor_values(m, pts))
    D = np.random.default_rng(7).choice([-1.0, 1.0], 200)
    a1 = solve_lstsq(A, v)
    a2 = solve_lstsq(D[:, None] * A, D * v)
    np.testing.assert_allclose(a1, a2, rtol=1e-11, atol=1e-12)
    G, h = A.T @ A, A.T @ v
    np.testing.assert_allclose(solve_cholesky(G, h), a1, rtol=1e-9, atol=1e-10)


def test_refit_requires_more_rows_than_core_entries():
    m = _model(rank=(2, 2, 2))
    pts = _pts(8, 100)
    with pytest.raises(ValueError):
        refit_core(m, pts, np.zeros(100), 8, seed=1)
    with pytest.raises(ValueError):
        sample_rows(1, 10, 11)


def test_residual_normal_vanishes_at_solution():
    m = _model(rank=(2, 2, 2), degree=(4, 4, 4))
    pts = _pts(9, 80)
    v = np.random.default_rng(9).standard_normal(80)
    G, h = normal_equations(m, pts, v)
    a = solve_cholesky(G, h)
    r = residual_normal(m, pts, v, a, chunk=13)
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(h)
    r0 = residual_normal(m, pts, v, np.zeros(m.R))
    np.testing.assert_allclose(r0, h, rtol=1e-12, atol=1e-13)


def test_evaluate_equals_full_expansion_and_design_rows():
    m = _model(lo=(0, 0, 0), hi=(4, 1, 1))
    pts = _pts(10, 400, (0, 0, 0), (4, 1, 1))
    f = evaluate(m, pts, chunk=37)
    np.testing.assert_allclose(f, evaluate_full_expansion(m, pts), rtol=1e-11, atol=1e-12)
    A = design_rows(factor_values(m, pts))
    np.testing.assert_allclose(f, A @ m.core.reshape(-1), rtol=1e-11, atol=1e-12)


def test_full_expansion_coefficients_definition():
    m = _model()
    beta = full_expansion_coefficients(m)
    ref = np.einsum("abc,ia,jb,kc->ijk", m.core, *m.coefs)
    np.testing.assert_allclose(beta, ref, atol=1e-13)


def test_grid_evaluation_matches_pointwise():
    m = _model()
    grid = (4, 3, 5)
    Y = evaluate_on_grid(m, grid)
    f = evaluate(m, grid_points(grid))
    np.testing.assert_allclose(Y.reshape(-1), f, rtol=1e-12, atol=1e-13)
    F = [legendre_orthonormal(grid_nodes(I), m.degree[k]) @ m.coefs[k] for k, I in enumerate(grid)]
    np.testing.assert_allclose(Y, tucker_full(m.core, F), atol=1e-13)


def test_tensor_grid_matches_pointwise_and_expansion():
    # arbitrary (unsorted, uneven) axes on a non-unit box, including a 1-point axis (a slice):
    # the mode-product form against eq. (1) point by point and against the full expansion
    m = _model(seed=3, rank=(3, 4, 2), degree=(5, 4, 6), lo=(0, -2, 1), hi=(4, 1, 3))
    rng = np.random.default_rng(7)
    gx, gy, gz = rng.uniform(0, 4, 5), rng.uniform(-2, 1, 1), rng.uniform(1, 3, 4)
    Y = evaluate_tensor_grid(m, gx, gy, gz)
    assert Y.shape == (5, 1, 4)
    P = np.stack(np.meshgrid(gx, gy, gz, indexing="ij"), axis=-1).reshape(-1, 3)
    np.testing.assert_allclose(Y.reshape(-1), evaluate(m, P), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Y.reshape(-1), evaluate_full_expansion(m, P), rtol=1e-11, atol=1e-12)
    # on the reference grid nodes it is the equispaced preview form
    grid = (4, 3, 5)
    g = [m.lo[k] + (grid_nodes(grid[k]) + 1) * (m.hi[k] - m.lo[k]) / 2 for k in range(3)]
    np.testing.assert_allclose(evaluate_tensor_grid(m, *g), evaluate_on_grid(m, grid), atol=1e-12)


def test_storage_accounting_and_csc():
    m = _model(rank=(3, 4, 2), degree=(5, 4, 6))
    nnz = sum(int((C != 0).sum()) for C in m.coefs)
    assert m.paper_bytes() == 8 * (24 + nnz)
    colptr, rows, vals = to_csc(m.coefs[1])
    assert colptr[-1] == np.count_nonzero(m.coefs[1])
    D = np.zeros_like(m.coefs[1])
    for j in range(D.shape[1]):
        D[rows[colptr[j]:colptr[j + 1]], j] = vals[colptr[j]:colptr[j + 1]]
    np.testing.assert_array_equal(D, m.coefs[1])
