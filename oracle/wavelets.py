"""Multiresolution wavelet basis W_{s,q} of Sec. 4.2 (oracle, test infrastructure): plain
numpy in FP64.

Sec. 4.2 approximates each singular vector in two spaces, the Legendre polynomials P_p and the
multiresolution wavelets W_{s,q} of resolution s and degree q, and keeps the approximation with
the smaller error.  The paper does not define W_{s,q} further.  Readings taken:

* W_{s,q} is the space of piecewise polynomials of degree <= q on the 2^s equal dyadic cells of
  [-1, 1] (dimension (q + 1) 2^s), with the multiwavelet basis of Alpert (1993): the global
  Legendre functions phi_0..phi_q, and for every level l = 0..s-1 and cell c = 0..2^l - 1 the
  q + 1 functions psi_{l,c,m}(t) = 2^(l/2) psi_m(2^l (t + 1) - 2c - 1) supported on that cell;
  all orthonormal under dt/2 on [-1, 1], like the Legendre functions;
* the mother wavelets psi_0..psi_q live on [-1, 1], are polynomials of degree <= q on [-1, 0)
  and on [0, 1], and are defined from the top down: psi_m is the unit-norm function of that
  space orthogonal to phi_0 .. phi_{q+m} (q + 1 + m vanishing moments) and to psi_{m+1} ..
  psi_q, which leaves one direction; its sign makes the largest coefficient of its right half,
  in the basis sqrt(2) phi_n(2x - 1), positive (the lowest n on ties);
* a point's cell at level l is floor((t + 1) 2^(l-1)), clamped to [0, 2^l - 1], so points on a
  cell boundary belong to the right-hand cell and t = 1 to the last cell;
* the basis of a mode holding both spaces (q <= p) is phi_0..phi_p followed by the detail
  functions psi_{l,c,m} in the order (l, c, m), so a coefficient column uses either the first
  p + 1 rows (a Legendre approximation) or rows 0..q and the detail rows (a wavelet one).
"""
from __future__ import annotations

import numpy as np

from .basis import legendre_orthonormal


def _half_gram(q: int):
    """Inner products <h_{half,n}, phi_i> for i = 0..2q under dt/2 on [-1, 1], with the
    orthonormal half-cell functions h_{L,n}(x) = sqrt(2) phi_n(2x + 1) on [-1, 0) and
    h_{R,n}(x) = sqrt(2) phi_n(2x - 1) on [0, 1]; columns (L, 0..q), (R, 0..q)."""
    xg, wg = np.polynomial.legendre.leggauss(2 * q + 2)    # exact for degree <= 4q + 3
    M = np.zeros((2 * q + 1, 2 * (q + 1)))
    for half, sgn in ((0, -1.0), (1, 1.0)):
        x = (xg + sgn) / 2.0                                # Gauss nodes mapped into the half
        h = np.sqrt(2.0) * legendre_orthonormal(xg, q)      # h_{half,n}(x): y = 2x -+ 1 = xg
        g = legendre_orthonormal(x, 2 * q)                  # phi_i(x)
        # int_half f dx/2 = (1/2) int_{-1}^{1} f(x(y)) dy/2 = (1/4) sum_k w_k f(x_k)
        M[:, half * (q + 1):(half + 1) * (q + 1)] = 0.25 * (g.T * wg) @ h
    return M


def mother_wavelets(q: int) -> np.ndarray:
    """(q + 1, 2, q + 1) array H: psi_m(x) = sqrt(2) sum_n H[m, half, n] phi_n(2x -+ 1)."""
    M = _half_gram(q)
    psi = [None] * (q + 1)
    for m in range(q, -1, -1):
        rows = [M[: q + m + 1]] + [psi[k][None, :] for k in range(m + 1, q + 1)]
        A = np.vstack(rows)                                  # 2q + 1 constraints, 2q + 2 unknowns
        _, _, Vt = np.linalg.svd(A)
        v = Vt[-1]
        right = v[q + 1:]
        if right[int(np.argmax(np.abs(right)))] < 0:
            v = -v
        psi[m] = v / np.linalg.norm(v)
    return np.stack([p.reshape(2, q + 1) for p in psi])


def detail_count(s: int, q: int) -> int:
    """Number of detail functions of W_{s,q}: (q + 1)(2^s - 1)."""
    return (q + 1) * ((1 << s) - 1)


def detail_values(t: np.ndarray, s: int, q: int, H: np.ndarray | None = None) -> np.ndarray:
    """(len(t), (q + 1)(2^s - 1)) values of psi_{l,c,m}(t) in the order (l, c, m)."""
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    if H is None:
        H = mother_wavelets(q)
    out = np.zeros((t.shape[0], detail_count(s, q)))
    for l in range(s):
        ncell = 1 << l
        c = np.clip(np.floor((t + 1.0) * ncell / 2.0), 0, ncell - 1).astype(np.int64)
        x = (t + 1.0) * ncell - 2.0 * c - 1.0
        right = x >= 0.0
        y = np.where(right, 2.0 * x - 1.0, 2.0 * x + 1.0)
        ph = legendre_orthonormal(y, q)                     # phi_n(y)
        half = right.astype(np.int64)
        vals = np.sqrt(2.0) * np.einsum("pn,pmn->pm", ph, H[:, half, :].transpose(1, 0, 2))
        vals *= 2.0 ** (l / 2.0)
        base = (q + 1) * (ncell - 1)
        for m in range(q + 1):
            out[np.arange(t.shape[0]), base + (q + 1) * c + m] = vals[:, m]
    return out


def mode_basis(t: np.ndarray, p: int, s: int = 0, q: int = 0) -> np.ndarray:
    """The basis of one mode at t: phi_0..phi_p, then the detail functions of W_{s,q}
    (none when s = 0)."""
    P = legendre_orthonormal(t, p)
    if s == 0:
        return P
    return np.hstack([P, detail_values(t, s, q)])


def wavelet_columns(p: int, s: int, q: int) -> np.ndarray:
    """Indices, in the mode basis, of the wavelet space W_{s,q}: phi_0..phi_q and the details."""
    return np.concatenate([np.arange(q + 1), p + 1 + np.arange(detail_count(s, q))])
