"""Pins of the oracle's Lasso-LARS sparse solver (Sec. 3, problem (5); ``oracle.lars``): the
optimality conditions of the Lasso at every event of the path, an independent coordinate-
descent Lasso solver at the path's regularisation values, the soft-threshold closed form on an
orthonormal design, the least-squares end of the path, exact recovery of sparse Legendre
combinations, and PRESS against brute-force leave-one-out."""
import numpy as np
import pytest

from oracle.basis import legendre_orthonormal
from oracle.interp import grid_nodes
from oracle.lars import lars_loo, lasso_lars_path
from oracle.sparsefit import fit_factor, press_bruteforce


def _design(seed, I=30, n=10):
    # correlated columns (column 1 close to column 0) so that the path has a drop event
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((I, n))
    X[:, 1] = X[:, 0] + 0.3 * rng.standard_normal(I)
    X /= np.linalg.norm(X, axis=0)
    return X, rng.standard_normal(I)


def _kkt(X, z, beta):
    """lambda and the worst violation of the Lasso optimality conditions for
    (1/2) ||z - X beta||^2 + lambda ||beta||_1 with lambda = max_j |x_j^T r|."""
    g = X.T @ (z - X @ beta)
    lam = float(np.max(np.abs(g)))
    nz = beta != 0
    viol = float(np.max(np.abs(g[nz] - lam * np.sign(beta[nz])))) if nz.any() else 0.0
    return lam, viol


def _lasso_cd(X, z, lam, iters=20000):
    """Cyclic coordinate descent on (1/2) ||z - X b||^2 + lam ||b||_1 (unit-norm columns)."""
    b = np.zeros(X.shape[1])
    r = z.copy()
    for _ in range(iters):
        bmax = 0.0
        for j in range(X.shape[1]):
            rho = X[:, j] @ r + b[j]
            nb = np.sign(rho) * max(abs(rho) - lam, 0.0)
            if nb != b[j]:
                r -= X[:, j] * (nb - b[j])
                bmax = max(bmax, abs(nb - b[j]))
                b[j] = nb
        if bmax < 1e-15:
            break
    return b


def test_path_satisfies_lasso_optimality_at_every_event():
    X, z = _design(0)
    events = lasso_lars_path(X, z, 10)
    assert "drop" in [e[2] for e in events]
    lam0 = float(np.max(np.abs(X.T @ z)))
    for A, beta, kind in events:
        lam, viol = _kkt(X, z, beta)
        assert viol <= 1e-10 * lam0
        assert set(np.nonzero(beta)[0]) <= set(A)          # non-zeros only in the active set


def test_path_matches_coordinate_descent_lasso():
    X, z = _design(0)
    events = lasso_lars_path(X, z, 10)
    kinds = [e[2] for e in events]
    picks = [1, 4, kinds.index("drop"), kinds.index("drop") + 1, len(events) - 2]
    for k in picks:
        beta = events[k][1]
        lam, _ = _kkt(X, z, beta)
        np.testing.assert_allclose(beta, _lasso_cd(X, z, lam), atol=1e-9)


def test_orthonormal_design_is_soft_thresholding():
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.standard_normal((40, 8)))[0]
    z = rng.standard_normal(40)
    events = lasso_lars_path(Q, z, 8)
    assert all(e[2] != "drop" for e in events)
    order = np.argsort(-np.abs(Q.T @ z), kind="stable")
    for k, (A, beta, kind) in enumerate(events[:8]):
        assert list(A) == list(order[: k + 1])
    for A, beta, kind in events[1:]:
        lam, _ = _kkt(Q, z, beta)
        cz = Q.T @ z
        np.testing.assert_allclose(beta, np.sign(cz) * np.maximum(np.abs(cz) - lam, 0.0), atol=1e-12)


def test_end_of_path_is_least_squares():
    X, z = _design(5, I=25, n=6)
    events = lasso_lars_path(X, z, 6)
    assert events[-1][2] == "end" and len(events[-1][0]) == 6
    np.testing.assert_allclose(events[-1][1], np.linalg.lstsq(X, z, rcond=None)[0], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("support", [[0], [3], [1, 6], [2, 5, 11]])
def test_lars_recovers_sparse_legendre_combination(support):
    Phi = legendre_orthonormal(grid_nodes(33), 15)
    c = np.zeros(16)
    c[support] = np.linspace(1.0, -0.6, len(support))
    S, coef, press = lars_loo(Phi, Phi @ c)
    assert sorted(S.tolist()) == sorted(support)
    got = np.zeros(16)
    got[S] = coef
    np.testing.assert_allclose(got, c, atol=1e-12)


def test_press_of_every_path_set_matches_bruteforce():
    rng = np.random.default_rng(9)
    Phi = legendre_orthonormal(grid_nodes(20), 9)
    z = np.sin(3 * grid_nodes(20)) + 0.05 * rng.standard_normal(20)
    S, coef, press = lars_loo(Phi, z)
    events = lasso_lars_path(Phi / np.linalg.norm(Phi, axis=0), z, min(10, 18))
    sets = [list(A) for A, _, _ in events][: len(press)]
    for A, pk in zip(sets, press):
        assert pk == pytest.approx(press_bruteforce(Phi[:, A], z), rel=1e-9)
    assert list(S) == sets[int(np.argmin(press))]


def test_fit_factor_with_lars_zero_column_and_shape():
    W = np.zeros((12, 3))
    W[:, 1] = legendre_orthonormal(grid_nodes(12), 4)[:, 2]
    C = fit_factor(W, grid_nodes(12), 6, solver="lars")
    assert C.shape == (7, 3)
    assert np.all(C[:, 0] == 0) and np.all(C[:, 2] == 0)
    np.testing.assert_allclose(C[:, 1], np.eye(7)[2], atol=1e-12)
