"""Pins of the oracle's 4-way form (d = 4: the space-time models of Sec. 6, eq. (1)-(2) with a
fourth factor): factor values and design rows by brute force, the Kronecker closed form of the
Gram on a full 4-D tensor grid, exact recovery of a planted core, the full least-squares
solution against an SVD-based solve, evaluation against a brute-force quadruple sum and the
full tensor-product expansion, ST-HOSVD exact recovery of a 4-way Tucker tensor, and
Algorithm 1 + 2 on a separable 4-D field."""
import numpy as np
import pytest

from datagen import random_model_parts, spacetime_f32
from oracle.basis import legendre_orthonormal
from oracle.interp import grid_nodes, grid_points
from oracle.lsq import design_rows, factor_values, normal_equations, refit_core, solve_lstsq
from oracle.model import Model
from oracle.pipeline import fit
from oracle.reconstruct import (evaluate, evaluate_full_expansion, evaluate_on_grid,
                                full_expansion_coefficients, rel_l2)
from oracle.sthosvd import st_hosvd, tucker_full


def _model(seed=0, rank=(2, 3, 2, 3), degree=(4, 5, 3, 6), lo=(-1,) * 4, hi=(1,) * 4):
    core, coefs = random_model_parts(seed, rank, degree)
    return Model(tuple(lo), tuple(hi), tuple(rank), tuple(degree), core, coefs)


def _pts(seed, n, lo=(-1,) * 4, hi=(1,) * 4):
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return lo + (hi - lo) * rng.random((n, 4))


def _legendre_by_hand(t, i):
    P = [1.0, t]
    for s in range(1, i):
        P.append(((2 * s + 1) * t * P[s] - s * P[s - 1]) / (s + 1))
    return np.sqrt(2 * i + 1) * P[i]


def test_factor_values_bruteforce_four_modes():
    lo, hi = (0, -1, 2, 0), (4, 1, 3, 10)
    m = _model(lo=lo, hi=hi)
    pts = _pts(1, 5, lo, hi)
    U = factor_values(m, pts)
    assert len(U) == 4
    for k in range(4):
        for q in range(5):
            xi = 2 * (pts[q, k] - lo[k]) / (hi[k] - lo[k]) - 1
            for j in range(m.rank[k]):
                s = sum(m.coefs[k][i, j] * _legendre_by_hand(xi, i) for i in range(m.degree[k] + 1))
                assert U[k][q, j] == pytest.approx(s, rel=1e-12, abs=1e-14)


def test_design_rows_four_modes_bruteforce_and_kron():
    m = _model()
    U = factor_values(m, _pts(2, 4))
    A = design_rows(U)
    r1, r2, r3, r4 = m.rank
    assert A.shape == (4, m.R)
    for q in range(4):
        for j1 in range(r1):
            for j2 in range(r2):
                for j3 in range(r3):
                    for j4 in range(r4):
                        j = ((j1 * r2 + j2) * r3 + j3) * r4 + j4
                        assert A[q, j] == pytest.approx(U[0][q, j1] * U[1][q, j2] * U[2][q, j3] * U[3][q, j4],
                                                        rel=1e-15)
        np.testing.assert_allclose(A[q], np.kron(np.kron(np.kron(U[0][q], U[1][q]), U[2][q]), U[3][q]),
                                   rtol=1e-15)


def test_gram_kronecker_closed_form_on_4d_tensor_grid():
    m = _model(rank=(2, 3, 2, 2), degree=(4, 5, 3, 4))
    grid = (4, 5, 3, 4)
    pts = grid_points(grid)
    assert pts.shape == (240, 4)
    G, _ = normal_equations(m, pts, np.zeros(pts.shape[0]), chunk=37)
    Gk = []
    for k, I in enumerate(grid):
        Uk = legendre_orthonormal(grid_nodes(I), m.degree[k]) @ m.coefs[k]
        Gk.append(Uk.T @ Uk)
    K = np.kron(np.kron(np.kron(Gk[0], Gk[1]), Gk[2]), Gk[3])
    np.testing.assert_allclose(G, K, rtol=1e-12, atol=1e-12)


def test_exact_recovery_of_planted_4way_core():
    m = _model(seed=4, rank=(3, 2, 3, 2), degree=(6, 6, 6, 6))
    pts = _pts(4, 2000)
    v = evaluate(m, pts)
    alpha, idx, _, _ = refit_core(m, pts, v, 300, seed=11)
    assert alpha.shape == (3, 2, 3, 2)
    np.testing.assert_allclose(alpha, m.core, rtol=1e-10, atol=1e-10)


def test_all_rows_equal_the_svd_least_squares_solution():
    m = _model(seed=5, rank=(2, 2, 3, 2), degree=(4, 4, 4, 4))
    pts = _pts(5, 400)
    v = np.random.default_rng(5).standard_normal(400)
    alpha, idx, _, _ = refit_core(m, pts, v, 400, seed=3)
    A = design_rows(factor_values(m, pts))
    a_qr = solve_lstsq(A, v)
    assert rel_l2(alpha.reshape(-1), a_qr) <= 100 * np.linalg.cond(A) ** 2 * 2.0 ** -53


def test_evaluate_four_modes_bruteforce_and_expansion():
    lo, hi = (0, 0, 0, -2), (4, 1, 1, 2)
    m = _model(seed=6, lo=lo, hi=hi)
    pts = _pts(6, 300, lo, hi)
    f = evaluate(m, pts, chunk=41)
    U = factor_values(m, pts[:3])
    for q in range(3):   # eq. (1) as a plain quadruple sum
        s = 0.0
        for j in np.ndindex(*m.rank):
            s += m.core[j] * U[0][q, j[0]] * U[1][q, j[1]] * U[2][q, j[2]] * U[3][q, j[3]]
        assert f[q] == pytest.approx(s, rel=1e-12, abs=1e-13)
    np.testing.assert_allclose(f, evaluate_full_expansion(m, pts), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(f, design_rows(factor_values(m, pts)) @ m.core.reshape(-1),
                               rtol=1e-11, atol=1e-12)
    beta = full_expansion_coefficients(m)
    np.testing.assert_allclose(beta, np.einsum("abcd,ia,jb,kc,ld->ijkl", m.core, *m.coefs), atol=1e-13)


def test_grid_evaluation_four_modes():
    m = _model(seed=7)
    grid = (3, 4, 2, 5)
    Y = evaluate_on_grid(m, grid)
    np.testing.assert_allclose(Y.reshape(-1), evaluate(m, grid_points(grid)), rtol=1e-12, atol=1e-13)
    F = [legendre_orthonormal(grid_nodes(I), m.degree[k]) @ m.coefs[k] for k, I in enumerate(grid)]
    np.testing.assert_allclose(Y, tucker_full(m.core, F), atol=1e-13)


def test_sthosvd_exact_recovery_four_way():
    rng = np.random.default_rng(8)
    dims, ranks = (9, 8, 7, 10), (3, 2, 4, 3)
    Q = [np.linalg.qr(rng.standard_normal((I, r)))[0] for I, r in zip(dims, ranks)]
    X = tucker_full(rng.standard_normal(ranks), Q)
    core, W, sig = st_hosvd(X, ranks)
    assert core.shape == ranks
    assert rel_l2(tucker_full(core, W), X) <= 1e-13
    for Wk in W:
        np.testing.assert_allclose(Wk.T @ Wk, np.eye(Wk.shape[1]), atol=1e-13)
    # truncating further: the error stays within the ST-HOSVD bound
    low = (2, 2, 3, 2)
    c2, W2, s2 = st_hosvd(X, low)
    err2 = np.linalg.norm(X - tucker_full(c2, W2)) ** 2
    bound = sum(float((s2[k][low[k]:] ** 2).sum()) for k in range(4))
    assert err2 <= bound * (1 + 1e-10) + 1e-20


def test_algorithms_1_and_2_on_a_separable_4d_field():
    # f = g1(x1) g2(x2) g3(x3) g4(x4) with polynomial g_k of degree <= 3, sampled at every node
    # of the 9^4 grid: the interpolation is exact at the nodes, the grid tensor has rank
    # (1,1,1,1), each singular vector is g_k at the nodes (up to scale), the sparse fit
    # recovers it in the degree-5 space, and the refit reproduces f to rounding
    grid = (9, 9, 9, 9)
    pts = grid_points(grid)
    g = [1.5 + pts[:, 0], 2 - pts[:, 1] ** 2, 1 + 0.5 * pts[:, 2] ** 3, 3 + pts[:, 3]]
    v = g[0] * g[1] * g[2] * g[3]
    m = fit(pts, v, (-1,) * 4, (1,) * 4, grid=grid, rank=(1, 1, 1, 1), degree=(5, 5, 5, 5),
            interp_fraction=1.0, n_samples=500, seed=2)
    assert rel_l2(evaluate(m, pts), v) < 1e-10
    rng = np.random.default_rng(9)
    off = rng.uniform(-1, 1, (500, 4))          # away from the nodes too
    v_off = (1.5 + off[:, 0]) * (2 - off[:, 1] ** 2) * (1 + 0.5 * off[:, 2] ** 3) * (3 + off[:, 3])
    assert rel_l2(evaluate(m, off), v_off) < 1e-10


def test_spacetime_workload_shape():
    w = spacetime_f32(n=1000, n_samples=100)
    assert w.pts.shape == (1000, 4) and w.pts.dtype == np.float32
    assert len(w.soa()) == 5
    assert np.all(w.pts[:, 3] >= 0) and np.all(w.pts[:, 3] <= 1)
    assert np.isfinite(w.vals).all() and float(np.std(w.vals)) > 0
