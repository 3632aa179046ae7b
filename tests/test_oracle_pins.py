"""Pins of the oracle's leverage scores (Sec. 5), of the corrector network's forward pass and
of the leave-one-out score at a node of leverage 1 (Sec. 3).  Each test names the mistake
in the oracle that it would catch."""
import math

import numpy as np
import pytest

from oracle import mlp
from oracle.lsq import leverage_scores
from oracle.sparsefit import omp_loo, press_bruteforce


# --- leverage scores --------------------------------------------------------------------

def test_leverage_of_orthonormal_columns_is_squared_row_norm():
    # For Q with orthonormal columns the left singular vectors span range(Q), so the
    # leverage of row i is ||Q[i, :]||^2.  Catches squaring the wrong factor (V or the
    # singular values) or summing over rows instead of columns.
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 6)))
    np.testing.assert_allclose(leverage_scores(Q), (Q ** 2).sum(axis=1), rtol=0, atol=1e-14)


def test_leverage_is_invariant_to_column_transforms_and_sums_to_rank():
    # leverage depends on range(A) only: A T has the same scores for any invertible T, and
    # they sum to rank(A).  Catches weighting by singular values (the scores of A and A T
    # would then differ) and keeping the directions of zero singular values (the sum would
    # exceed the rank).
    rng = np.random.default_rng(12)
    A = rng.standard_normal((50, 5))
    T = rng.standard_normal((5, 5)) + 5 * np.eye(5)
    la = leverage_scores(A)
    np.testing.assert_allclose(leverage_scores(A @ T), la, atol=1e-12)
    assert la.sum() == pytest.approx(5.0, abs=1e-12)
    assert la.min() >= -1e-15 and la.max() <= 1 + 1e-12
    # rank 3 design with 6 columns: columns 4..6 repeat combinations of columns 1..3
    B = rng.standard_normal((50, 3))
    B6 = np.hstack([B, B @ rng.standard_normal((3, 3))])
    lb = leverage_scores(B6)
    assert lb.sum() == pytest.approx(3.0, abs=1e-10)
    np.testing.assert_allclose(lb, leverage_scores(B), atol=1e-10)


def test_leverage_is_the_hat_matrix_diagonal():
    # for full column rank, h_ii = a_i^T (A^T A)^-1 a_i (the hat matrix of the least-squares
    # fit); written here through a linear solve, not an SVD
    rng = np.random.default_rng(13)
    A = rng.standard_normal((30, 4)) * np.array([1.0, 10.0, 0.1, 3.0])
    hat = np.einsum("ij,ij->i", A, np.linalg.solve(A.T @ A, A.T).T)
    np.testing.assert_allclose(leverage_scores(A), hat, rtol=1e-11)


def test_isolated_unit_row_has_leverage_one():
    # a row that alone carries a column (no other row can replace it) has leverage 1, and
    # the other rows then carry the rest.  Catches a normalisation by R/N or by the row count.
    rng = np.random.default_rng(14)
    A = np.zeros((20, 3))
    A[:, :2] = rng.standard_normal((20, 2))
    A[7, 2] = 2.5
    lev = leverage_scores(A)
    assert lev[7] == pytest.approx(1.0, abs=1e-13)
    assert lev.sum() == pytest.approx(3.0, abs=1e-12)
    assert np.all(leverage_scores(np.zeros((4, 2))) == 0.0)


# --- corrector network forward pass -----------------------------------------------------

def _hand_net():
    # 1 -> 2 -> 2 -> 1 network chosen so that every pre-activation is 0 or +-ln 3, where
    # SiLU is known exactly: s(0) = 0, s(ln 3) = (3/4) ln 3, s(-ln 3) = -(1/4) ln 3
    L = math.log(3.0)
    p = {"W1": np.array([[L / 2], [-L]]), "b1": np.array([0.0, L]),
         "W2": np.array([[2.0, 2.0], [1.0, 3.0]]), "b2": np.array([-L, L]),
         "W3": np.array([[5.0, 7.0]]), "b3": np.array([0.25])}
    return p, L


def test_mlp_forward_matches_hand_computed_value():
    # x = 2: z1 = (L, -L), a1 = (3L/4, -L/4); z2 = W2 a1 + b2 = (0, L), a2 = (0, 3L/4);
    # y = 5 * 0 + 7 * 3L/4 + 1/4.  A transposed W2 gives z2 = (L/4, 7L/4); a dropped b2 gives
    # z2 = (L, 0) and y = 15L/4 + 1/4; a dropped b1 or b3, or the sigmoid in place of SiLU,
    # also changes y.
    p, L = _hand_net()
    y, (x, z1, a1, z2, a2) = mlp.forward(p, np.array([[2.0]]))
    np.testing.assert_allclose(z1[0], [L, -L], rtol=1e-15)
    np.testing.assert_allclose(a1[0], [0.75 * L, -0.25 * L], rtol=1e-15)
    np.testing.assert_allclose(z2[0], [0.0, L], atol=1e-15)
    np.testing.assert_allclose(a2[0], [0.0, 0.75 * L], atol=1e-15)
    assert y[0] == pytest.approx(21.0 * L / 4.0 + 0.25, rel=1e-15)


def test_mlp_forward_is_row_independent_and_shaped():
    # a batch is evaluated row by row: the value of a row does not depend on its neighbours
    p, L = _hand_net()
    y, _ = mlp.forward(p, np.array([[0.0], [2.0], [1.0]]))
    assert y.shape == (3,)
    assert y[1] == pytest.approx(21.0 * L / 4.0 + 0.25, rel=1e-15)
    y1, _ = mlp.forward(p, np.array([[1.0]]))
    assert y[2] == pytest.approx(y1[0], rel=1e-15)


# --- leave-one-out score at a node of leverage 1 ------------------------------------------

def test_press_is_infinite_at_a_node_of_leverage_one():
    # column 1 is non-zero at node 3 only: once it is in the support the fit reproduces that
    # node exactly and its hat-matrix diagonal is 1, so its leave-one-out residual is 0/0.
    # The reading taken scores such a support +inf (no finite number, no NaN).
    Phi = np.array([[1.0, 0.0], [1.0, 0.0], [1.0, 0.0], [1.0, 1.0], [1.0, 0.0]])
    z = np.array([1.0, 1.1, 0.9, 5.0, 1.0])
    S, c, press = omp_loo(Phi, z)
    # column 1 has the larger normalised correlation (4.95 / 1 against 9.0 / sqrt(5))
    assert int(S[0]) == 1 and len(press) == 2
    assert press == [np.inf, np.inf]
    # every size scores +inf, so the first (smallest) support is kept
    assert len(S) == 1 and c[0] == pytest.approx(5.0)
    # a design without such a node keeps finite scores that equal brute-force refits
    Phi2 = np.array([[1.0, -1.0], [1.0, -0.5], [1.0, 0.0], [1.0, 0.5], [1.0, 1.0]])
    _, _, press2 = omp_loo(Phi2, z)
    assert all(np.isfinite(press2))
    assert press2[-1] == pytest.approx(press_bruteforce(Phi2, z), rel=1e-12)
