"""Core re-estimation by randomized least squares (oracle, test infrastructure).

Sec. 5 rewrites eq. (1) as u~(y) = sum_j alpha_j w_j(y) with w_j = prod_k w^(k)_{j_k} and
R = r1 ... r_d (d = 3, or 4 for the space-time form of Sec. 6), and re-estimates the core from the original scattered data by the regression
eq. (6): alpha^ = argmin ||u - W alpha||^2, W[q, j] = w_j(y^q).  Algorithm 2 solves it on a
sketch: rows of W and u are sign-flipped (D), mixed (FFT) and S > R of them are sampled
uniformly, and step 5 solves the sampled problem exactly.

Readings taken here:
* the core is vectorised in C order, j = (j1 r2 + j2) r3 + j3 (and j r4 + j4 for d = 4);
* the hot path samples M rows of W directly (no mixing).  D alone changes nothing, since
  (DW)^T (DW) = W^T W; the mixed variant is a separate, later row;
* step 5 is read as min_alpha ||S W alpha - S u||^2 (the printed formula drops alpha) and is
  solved through the normal equations G alpha = h, G = A^T A, h = A^T v, by a Cholesky
  factorisation; numpy's lstsq (SVD based) serves as an independent truth check.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .basis import to_reference
from .model import Model
from .sampler import STREAM_LS, sample_without_replacement
from .wavelets import mode_basis


def factor_values(model: Model, pts: np.ndarray):
    """[U_k (m, r_k)] for k = 1..d: U_k[q, j] = w^(k)_j(y^q_k) = sum_i C_k[i, j] phi_i(xi^q_k)
    (eq. (2)) over the mode's basis (Legendre, plus wavelet details when the model has them);
    pts has one column per mode."""
    pts = np.asarray(pts, dtype=np.float64)
    out = []
    for k in range(len(model.rank)):
        xi = to_reference(pts[:, k], model.lo[k], model.hi[k])
        out.append(mode_basis(xi, model.degree[k], *model.mode_wavelet(k)) @ model.coefs[k])
    return out


def design_rows(U) -> np.ndarray:
    """A[q, j] = prod_k U_k[q, j_k], j = (..((j1 r2 + j2) r3 + j3)..) r_d + j_d: the rows of W in
    eq. (6), each the Kronecker product of the point's factor rows in mode order."""
    A = np.asarray(U[0], np.float64)
    m = A.shape[0]
    for Uk in U[1:]:
        A = (A[:, :, None] * np.asarray(Uk, np.float64)[:, None, :]).reshape(m, -1)
    return A


def normal_equations(model: Model, pts: np.ndarray, v: np.ndarray, chunk: int = 4096):
    """G = A^T A and h = A^T v over the given rows, accumulated over point batches."""
    R = model.R
    G = np.zeros((R, R), dtype=np.float64)
    h = np.zeros(R, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    for s in range(0, pts.shape[0], chunk):
        A = design_rows(factor_values(model, pts[s:s + chunk]))
        G += A.T @ A
        h += A.T @ v[s:s + chunk]
    return G, h


def solve_cholesky(G: np.ndarray, h: np.ndarray) -> np.ndarray:
    """alpha = G^-1 h by Cholesky (LAPACK potrf/potrs through scipy)."""
    c, low = scipy.linalg.cho_factor(G, lower=True, check_finite=True)
    return scipy.linalg.cho_solve((c, low), h)


def solve_lstsq(A: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Least-squares solution by numpy's SVD-based lstsq (truth check for the normal equations)."""
    return np.linalg.lstsq(A, v, rcond=None)[0]


def sample_rows(seed: int, n: int, m: int) -> np.ndarray:
    """The M least-squares rows: uniform, without replacement, sorted (stream 2)."""
    if not (0 < m <= n):
        raise ValueError("need 0 < M <= N")
    return sample_without_replacement(seed, STREAM_LS, n, m)


def refit_core(model: Model, pts: np.ndarray, vals: np.ndarray, n_samples: int, seed: int,
               chunk: int = 4096):
    """Algorithm 2 with uniform row sampling: returns (alpha (r1, .., r_d), rows, G, h)."""
    if n_samples <= model.R:
        raise ValueError("Algorithm 2 needs more sampled rows than core entries (S > R)")
    idx = sample_rows(seed, pts.shape[0], n_samples)
    G, h = normal_equations(model, pts[idx], np.asarray(vals, np.float64)[idx], chunk)
    alpha = solve_cholesky(G, h)
    return alpha.reshape(model.rank), idx, G, h


def residual_normal(model: Model, pts: np.ndarray, v: np.ndarray, alpha: np.ndarray,
                    chunk: int = 4096) -> np.ndarray:
    """A^T (v - A alpha): the normal-equations residual used by iterative refinement."""
    r = np.zeros(model.R, dtype=np.float64)
    a = np.asarray(alpha, np.float64).reshape(-1)
    for s in range(0, pts.shape[0], chunk):
        A = design_rows(factor_values(model, pts[s:s + chunk]))
        r += A.T @ (np.asarray(v[s:s + chunk], np.float64) - A @ a)
    return r


def leverage_scores(A: np.ndarray) -> np.ndarray:
    """Leverage of every row of A (Sec. 5): the squared row norms of the left singular
    vectors that span the column space of A, i.e. those whose singular value exceeds
    max(m, n) * eps * sigma_max.  They lie in [0, 1] and sum to rank(A)."""
    A = np.asarray(A, np.float64)
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros(A.shape[0])
    keep = s > max(A.shape) * np.finfo(np.float64).eps * s[0]
    Uk = U[:, keep]
    return (Uk * Uk).sum(axis=1)
