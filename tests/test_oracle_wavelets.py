"""Pins of the oracle's multiresolution wavelet space W_{s,q} (Sec. 4.2; ``oracle.wavelets``)
and of the per-column choice between P_p and W_{s,q} in Algorithm 1: the Haar closed form at
q = 0 (mother and every dilated, translated detail function), orthonormality of the whole basis
by Gauss quadrature cell by cell, the vanishing moments that define the mother wavelets, their
even/odd symmetry, reproduction of arbitrary piecewise polynomials on the 2^s cells, the choice
of the smaller leave-one-out error, and the model forms (factor values, full expansion, grid,
exact recovery of a planted core) with wavelet factors."""
import numpy as np
import pytest

from datagen import random_model_parts
from oracle.basis import legendre_orthonormal
from oracle.interp import grid_nodes, grid_points
from oracle.lsq import design_rows, factor_values, refit_core
from oracle.model import Model
from oracle.reconstruct import evaluate, evaluate_full_expansion, evaluate_on_grid
from oracle.sparsefit import fit_factor_choice
from oracle.sthosvd import tucker_full
from oracle.wavelets import (detail_count, detail_values, mode_basis, mother_wavelets,
                             wavelet_columns)


def _cell_quadrature(s, npts):
    """Gauss nodes and dt/2 weights on every one of the 2^s cells of [-1, 1]."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    ts, ws = [], []
    h = 2.0 / (1 << s)
    for c in range(1 << s):
        a = -1.0 + c * h
        ts.append(a + (xg + 1.0) * h / 2.0)
        ws.append(wg * h / 4.0)        # dt/2 over a cell of width h: (h/2) (1/2) sum w
    return np.concatenate(ts), np.concatenate(ws)


def test_haar_at_degree_zero():
    H = mother_wavelets(0)
    np.testing.assert_allclose(np.sqrt(2) * H[0, :, 0], [-1.0, 1.0], atol=1e-15)
    s = 3
    t = np.random.default_rng(0).uniform(-1, 1, 500)
    D = detail_values(t, s, 0)
    col = 0
    for l in range(s):
        for c in range(1 << l):
            a, w = -1.0 + c * 2.0 / (1 << l), 2.0 / (1 << l)
            inside = (t >= a) & (t < a + w)
            ref = np.where(inside, np.where(t < a + w / 2, -1.0, 1.0), 0.0) * 2.0 ** (l / 2)
            np.testing.assert_allclose(D[:, col], ref, atol=1e-14)
            col += 1


@pytest.mark.parametrize("s,q", [(1, 0), (2, 1), (3, 2), (3, 3), (2, 5), (4, 3)])
def test_basis_is_orthonormal(s, q):
    t, w = _cell_quadrature(s, q + 2)
    B = mode_basis(t, q, s, q)
    assert B.shape[1] == (q + 1) << s
    np.testing.assert_allclose((B * w[:, None]).T @ B, np.eye(B.shape[1]), atol=1e-12)


@pytest.mark.parametrize("q", [0, 1, 2, 3, 5, 7])
def test_mother_wavelet_moments_and_parity(q):
    H = mother_wavelets(q)
    t, w = _cell_quadrature(1, 2 * q + 2)
    Psi = detail_values(t, 1, q, H)                     # level 0: the mother wavelets on [-1, 1]
    Phi = legendre_orthonormal(t, 2 * q + 1)
    Mom = (Psi * w[:, None]).T @ Phi                    # <psi_m, phi_i>
    for m in range(q + 1):
        np.testing.assert_allclose(Mom[m, : q + m + 1], 0.0, atol=1e-12)
    tt = np.linspace(0.01, 0.99, 37)
    for m in range(q + 1):
        a = detail_values(tt, 1, q, H)[:, m]
        b = detail_values(-tt, 1, q, H)[:, m]
        assert np.allclose(a, b, atol=1e-12) or np.allclose(a, -b, atol=1e-12)


@pytest.mark.parametrize("s,q", [(2, 1), (3, 3), (4, 2)])
def test_basis_reproduces_piecewise_polynomials(s, q):
    rng = np.random.default_rng(s * 10 + q)
    coef = rng.standard_normal((1 << s, q + 1))
    t = rng.uniform(-1, 1, 4000)
    h = 2.0 / (1 << s)
    c = np.clip(np.floor((t + 1) / h), 0, (1 << s) - 1).astype(int)
    local = (t + 1 - c * h) / h * 2 - 1
    f = np.einsum("pn,pn->p", legendre_orthonormal(local, q), coef[c])
    B = mode_basis(t, q, s, q)
    a, *_ = np.linalg.lstsq(B, f, rcond=None)
    assert np.linalg.norm(B @ a - f) <= 1e-11 * np.linalg.norm(f)


def test_choice_keeps_the_smaller_leave_one_out_error():
    nodes = grid_nodes(64)
    p, s, q = 12, 3, 2
    W = np.stack([1 + nodes - 0.5 * nodes ** 3,                    # a polynomial: P_p exact
                  np.where(nodes < 0.25, -1.0, 2.0),               # a step at a cell edge
                  np.exp(-nodes ** 2)], axis=1)
    C = fit_factor_choice(W, nodes, p, s, q)
    assert C.shape == (p + 1 + detail_count(s, q), 3)
    assert np.all(C[p + 1:, 0] == 0) and np.any(C[: p + 1, 0] != 0)      # Legendre kept (tie)
    assert np.any(C[p + 1:, 1] != 0) and np.all(C[q + 1: p + 1, 1] == 0)  # wavelet kept
    B = mode_basis(nodes, p, s, q)
    np.testing.assert_allclose(B @ C[:, 0], W[:, 0], atol=1e-12)
    np.testing.assert_allclose(B @ C[:, 1], W[:, 1], atol=1e-12)
    assert set(np.nonzero(C[:, 1])[0]) <= set(wavelet_columns(p, s, q).tolist())


def _wmodel(seed, rank=(3, 2, 3), degree=(7, 6, 8), wav=((2, 3), (3, 1), (1, 2))):
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(rank)
    coefs = []
    for k in range(3):
        n = degree[k] + 1 + detail_count(*wav[k])
        C = rng.standard_normal((n, rank[k])) * (rng.random((n, rank[k])) < 0.5)
        C[0] += 1.0
        coefs.append(C / np.sqrt(n))
    return Model((-1.0, 0.0, 2.0), (1.0, 3.0, 4.0), rank, degree, core, coefs, wavelet=wav)


def test_wavelet_model_forms_agree():
    m = _wmodel(1)
    rng = np.random.default_rng(2)
    pts = np.stack([rng.uniform(-1, 1, 300), rng.uniform(0, 3, 300), rng.uniform(2, 4, 300)], axis=1)
    U = factor_values(m, pts)
    for k in range(3):
        xi = 2 * (pts[:, k] - m.lo[k]) / (m.hi[k] - m.lo[k]) - 1
        np.testing.assert_allclose(U[k], mode_basis(xi, m.degree[k], *m.wavelet[k]) @ m.coefs[k], atol=1e-14)
    f = evaluate(m, pts)
    np.testing.assert_allclose(f, evaluate_full_expansion(m, pts), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(f, design_rows(U) @ m.core.reshape(-1), rtol=1e-11, atol=1e-12)
    grid = (5, 4, 6)
    Y = evaluate_on_grid(m, grid)
    F = [mode_basis(grid_nodes(I), m.degree[k], *m.wavelet[k]) @ m.coefs[k] for k, I in enumerate(grid)]
    np.testing.assert_allclose(Y, tucker_full(m.core, F), atol=1e-13)


def test_planted_core_recovered_with_wavelet_factors():
    m = _wmodel(3)
    rng = np.random.default_rng(4)
    pts = np.stack([rng.uniform(-1, 1, 3000), rng.uniform(0, 3, 3000), rng.uniform(2, 4, 3000)], axis=1)
    alpha, _, _, _ = refit_core(m, pts, evaluate(m, pts), 400, seed=5)
    np.testing.assert_allclose(alpha, m.core, rtol=1e-9, atol=1e-9)
