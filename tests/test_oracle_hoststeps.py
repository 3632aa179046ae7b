"""Pins of the oracle's host-side steps: interpolation onto the grid, ST-HOSVD and the
sparse (OMP + leave-one-out) Legendre fit."""
import numpy as np
import pytest

from oracle.basis import legendre_orthonormal
from oracle.interp import grid_nodes, grid_points, idw_to_grid
from oracle.sparsefit import fit_factor, omp_loo, press_bruteforce
from oracle.sthosvd import fix_signs, mode_product, st_hosvd, tucker_full, unfold, ranks_for_precision


# ----------------------------------------------------------------------------- interpolation

def test_grid_nodes_equispaced_with_endpoints():
    g = grid_nodes(5)
    np.testing.assert_allclose(g, [-1, -0.5, 0, 0.5, 1], atol=0)
    P = grid_points((2, 3, 4))
    assert P.shape == (24, 3)
    np.testing.assert_allclose(P[1], [-1, -1, -1 + 2 / 3])   # last mode fastest


def _idw_bruteforce(xi, v, nodes, k, power):
    out = np.empty(nodes.shape[0])
    for i, x in enumerate(nodes):
        d = np.sqrt(((xi - x) ** 2).sum(axis=1))
        nn = np.argsort(d, kind="stable")[:k]
        if d[nn[0]] == 0:
            out[i] = v[nn[0]]
            continue
        w = 1.0 / d[nn] ** power
        out[i] = (w * v[nn]).sum() / w.sum()
    return out


def test_idw_matches_bruteforce():
    rng = np.random.default_rng(0)
    xi = rng.uniform(-1, 1, (60, 3))
    v = rng.standard_normal(60)
    T = idw_to_grid(xi, v, (4, 5, 3), k=8, power=2.0)
    ref = _idw_bruteforce(xi, v, grid_points((4, 5, 3)), 8, 2.0)
    np.testing.assert_allclose(T.reshape(-1), ref, rtol=1e-13, atol=1e-14)


def test_idw_reproduces_constants_and_is_exact_at_nodes():
    rng = np.random.default_rng(1)
    xi = rng.uniform(-1, 1, (200, 3))
    T = idw_to_grid(xi, np.full(200, 3.25), (6, 6, 6))
    np.testing.assert_allclose(T, 3.25, rtol=1e-14)
    # plant data points exactly on two grid nodes
    nodes = grid_points((6, 6, 6))
    xi2 = np.vstack([xi, nodes[[7, 100]]])
    v2 = np.concatenate([rng.standard_normal(200), [11.0, -4.0]])
    T2 = idw_to_grid(xi2, v2, (6, 6, 6)).reshape(-1)
    assert T2[7] == 11.0 and T2[100] == -4.0


# ----------------------------------------------------------------------------- ST-HOSVD

def _random_orthonormal(rng, n, r):
    Q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return Q


def test_sthosvd_recovers_exact_low_rank():
    rng = np.random.default_rng(2)
    r = (3, 4, 2)
    G = rng.standard_normal(r)
    Q = [_random_orthonormal(rng, n, rk) for n, rk in zip((10, 12, 9), r)]
    X = tucker_full(G, Q)
    core, W, _ = st_hosvd(X, r)
    Xr = tucker_full(core, W)
    assert np.linalg.norm(Xr - X) / np.linalg.norm(X) < 1e-13
    for k in range(3):
        np.testing.assert_allclose(W[k].T @ W[k], np.eye(r[k]), atol=1e-13)
        # same column space as the planted factor
        P = W[k] @ W[k].T
        assert np.linalg.norm(P @ Q[k] - Q[k]) < 1e-12


def test_sthosvd_error_bound_and_signs():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((8, 7, 6))
    r = (3, 3, 2)
    core, W, sig = st_hosvd(X, r)
    err2 = np.linalg.norm(X - tucker_full(core, W)) ** 2
    bound = sum((s[rk:] ** 2).sum() for s, rk in zip(sig, r))
    assert err2 <= bound * (1 + 1e-12)
    for Wk in W:
        for j in range(Wk.shape[1]):
            i = np.argmax(np.abs(Wk[:, j]))
            assert Wk[i, j] > 0
    # full ranks reproduce the tensor exactly
    core_f, W_f, _ = st_hosvd(X, X.shape)
    np.testing.assert_allclose(tucker_full(core_f, W_f), X, atol=1e-12)


def test_mode_product_and_unfold_definitions():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3, 4, 5))
    M = rng.standard_normal((2, 4))
    Y = mode_product(X, M, 1)
    ref = np.einsum("ajc,bj->abc", X, M)
    np.testing.assert_allclose(Y, ref, atol=1e-14)
    assert unfold(X, 2).shape == (5, 12)
    np.testing.assert_allclose(unfold(X, 2)[:, 0], X[0, 0, :])


def test_ranks_for_precision_meets_eps():
    rng = np.random.default_rng(5)
    G = rng.standard_normal((3, 3, 3))
    X = tucker_full(G, [_random_orthonormal(rng, 9, 3) for _ in range(3)])
    X = X + 1e-6 * rng.standard_normal(X.shape)
    r = ranks_for_precision(X, 1e-3)
    assert r == (3, 3, 3)
    core, W, _ = st_hosvd(X, r)
    assert np.linalg.norm(X - tucker_full(core, W)) <= 1e-3 * np.linalg.norm(X)


def test_fix_signs():
    U = np.array([[0.1, -0.9], [-0.8, 0.2]])
    F = fix_signs(U)
    np.testing.assert_allclose(F, [[-0.1, 0.9], [0.8, -0.2]])


# ----------------------------------------------------------------------------- sparse fit

@pytest.mark.parametrize("support", [[0], [3, 11], [1, 6, 14]])
def test_omp_recovers_sparse_legendre_combination(support):
    nodes = grid_nodes(32)
    Phi = legendre_orthonormal(nodes, 15)
    c = np.zeros(16)
    rng = np.random.default_rng(len(support))
    c[support] = rng.uniform(0.5, 2.0, len(support)) * rng.choice([-1, 1], len(support))
    z = Phi @ c
    S, coef, press = omp_loo(Phi, z)
    assert sorted(S.tolist()) == sorted(support)
    full = np.zeros(16)
    full[S] = coef
    np.testing.assert_allclose(full, c, atol=1e-12)


def test_press_matches_bruteforce_leave_one_out():
    rng = np.random.default_rng(6)
    nodes = grid_nodes(20)
    Phi = legendre_orthonormal(nodes, 9)
    z = np.sin(2.5 * nodes) + 0.01 * rng.standard_normal(20)
    S, coef, press = omp_loo(Phi, z)
    # recompute the whole PRESS path by brute-force refits on each prefix of the selection order
    order = []
    r = z.copy()
    colnorm = np.linalg.norm(Phi, axis=0)
    for t in range(len(press)):
        score = np.abs(Phi.T @ r) / colnorm
        score[order] = -1
        order.append(int(np.argmax(score)))
        c, *_ = np.linalg.lstsq(Phi[:, order], z, rcond=None)
        r = z - Phi[:, order] @ c
        assert press[t] == pytest.approx(press_bruteforce(Phi[:, order], z), rel=1e-9)
    assert len(S) == int(np.argmin(press)) + 1


def test_fit_factor_zero_column_and_shape():
    nodes = grid_nodes(16)
    W = np.zeros((16, 2))
    W[:, 1] = legendre_orthonormal(nodes, 5)[:, 2]
    C = fit_factor(W, nodes, 5)
    assert C.shape == (6, 2)
    assert np.count_nonzero(C[:, 0]) == 0
    np.testing.assert_allclose(C[:, 1], np.eye(6)[2], atol=1e-13)
