"""Reference coordinates and the orthonormal Legendre basis (oracle, test infrastructure).

Sec. 2 asks for approximation spaces with an orthonormal basis; Sec. 4.2 names the space
of Legendre polynomials of degree p.  Reading taken: phi_m(t) = sqrt(2m+1) P_m(t),
m = 0..p, orthonormal on [-1,1] under the uniform probability measure dt/2, so each mode
has n = p+1 functions.  Coordinates are mapped affinely from the configured box onto
[-1,1] (the paper leaves the mapping unstated).
"""
from __future__ import annotations

import numpy as np


def to_reference(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """xi = 2 (x - lo) / (hi - lo) - 1, elementwise, float64."""
    x = np.asarray(x, dtype=np.float64)
    return 2.0 * (x - lo) / (hi - lo) - 1.0


def legendre_P(t: np.ndarray, p: int) -> np.ndarray:
    """Classical Legendre polynomials P_0..P_p at t, shape (len(t), p+1).

    Bonnet's three-term recurrence: (m+1) P_{m+1} = (2m+1) t P_m - m P_{m-1}.
    """
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    out = np.empty((t.shape[0], p + 1), dtype=np.float64)
    out[:, 0] = 1.0
    if p >= 1:
        out[:, 1] = t
    for m in range(1, p):
        out[:, m + 1] = ((2 * m + 1) * t * out[:, m] - m * out[:, m - 1]) / (m + 1)
    return out


def legendre_orthonormal(t: np.ndarray, p: int) -> np.ndarray:
    """phi_m(t) = sqrt(2m+1) P_m(t), m = 0..p; shape (len(t), p+1)."""
    scale = np.sqrt(2.0 * np.arange(p + 1) + 1.0)
    return legendre_P(t, p) * scale[None, :]
