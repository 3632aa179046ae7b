"""Evaluation of the functional sparse Tucker model (oracle, test infrastructure).

Sec. 6: reconstruction needs only the evaluation of the basis functions at the points of
interest, followed by eq. (1).  Two independent forms are provided so that each pins the
other: the Tucker form of eq. (1) and the full tensor-product expansion of Sec. 2 with
beta = alpha x_1 C_1 x_2 C_2 x_3 C_3.
"""
from __future__ import annotations

import numpy as np

from .basis import to_reference
from .interp import grid_nodes
from .lsq import factor_values
from .model import Model
from .sthosvd import mode_product
from .wavelets import mode_basis


def _contract_rows(rows, T) -> np.ndarray:
    """sum over (a, b, ..) of T[a, b, ..] rows[0][q, a] rows[1][q, b] .. for every q."""
    idx = "abcd"[:len(rows)]
    spec = ",".join("q" + c for c in idx) + "," + idx + "->q"
    return np.einsum(spec, *rows, T, optimize=True)


def evaluate(model: Model, pts: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """u~(y^q) = sum_{j1 .. jd} alpha_{j1 .. jd} U1[q,j1] .. Ud[q,jd]  (eq. (1), d = 3 or 4)."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.empty(pts.shape[0], dtype=np.float64)
    core = np.asarray(model.core, np.float64)
    for s in range(0, pts.shape[0], chunk):
        out[s:s + chunk] = _contract_rows(factor_values(model, pts[s:s + chunk]), core)
    return out


def full_expansion_coefficients(model: Model) -> np.ndarray:
    """beta (n1, .., nd) of the tensor-product expansion equal to the Tucker model (n_k: the size
    of the mode's basis)."""
    beta = np.asarray(model.core, np.float64)
    for k in range(len(model.rank)):
        beta = mode_product(beta, model.coefs[k], k)
    return beta


def evaluate_full_expansion(model: Model, pts: np.ndarray) -> np.ndarray:
    """u(y) = sum_{i1 .. id} beta_{i1 .. id} phi_i1(y1) .. phi_id(yd)  (Sec. 2)."""
    beta = full_expansion_coefficients(model)
    pts = np.asarray(pts, dtype=np.float64)
    P = [mode_basis(to_reference(pts[:, k], model.lo[k], model.hi[k]), model.degree[k], *model.mode_wavelet(k))
         for k in range(len(model.rank))]
    return _contract_rows(P, beta)


def evaluate_on_grid(model: Model, grid) -> np.ndarray:
    """Reconstruction on an equispaced reference grid by mode products (preview form):
    alpha x_1 (Phi_1 C_1) x_2 (Phi_2 C_2) .. x_d (Phi_d C_d)."""
    Y = np.asarray(model.core, np.float64)
    for k in range(len(grid)):
        F = mode_basis(grid_nodes(grid[k]), model.degree[k], *model.mode_wavelet(k)) @ model.coefs[k]
        Y = mode_product(Y, F, k)
    return Y


def evaluate_tensor_grid(model: Model, gx, gy, gz) -> np.ndarray:
    """Reconstruction on the tensor grid gx x gy x gz of physical coordinates (Sec. 6 preview
    form): alpha x_1 U1 x_2 U2 x_3 U3 with U_k = Phi_k(xi_k(g_k)) C_k, the factor functions of
    eq. (2) at the grid lines of mode k.  Returns an (n1, n2, n3) array."""
    Y = np.asarray(model.core, np.float64)
    for k, g in enumerate((gx, gy, gz)):
        t = to_reference(np.asarray(g, np.float64), model.lo[k], model.hi[k])
        Y = mode_product(Y, mode_basis(t, model.degree[k], *model.mode_wavelet(k)) @ model.coefs[k], k)
    return Y


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2."""
    x = np.asarray(x, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
