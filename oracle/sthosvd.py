"""Sequentially truncated HOSVD at fixed ranks (oracle, test infrastructure).

Sec. 4.1 decomposes the grid tensor U ~ alpha x_1 W1 x_2 W2 x_3 W3 with TuckerMPI, a
parallel implementation of ST-HOSVD (Vannieuwenhoven, Vandebril, Meerbergen 2012).  The
sequential algorithm: for k = 1..d, take the mode-k unfolding of the current (already
partly truncated) tensor, keep its r_k leading left singular vectors as W_k, and replace
the tensor by its mode-k product with W_k^T.  What remains is the core.

Readings taken (the paper fixes none of them): modes are processed in the order 1, 2, 3;
singular vectors come from numpy's SVD (LAPACK) in descending singular-value order; the
sign of each vector is fixed so that its largest-magnitude entry is positive (ties go to
the lowest index).  The precision-driven rank choice of the paper is offered by
``ranks_for_precision`` and is not used by the fixed-rank workloads.
"""
from __future__ import annotations

import numpy as np


def unfold(Y: np.ndarray, k: int) -> np.ndarray:
    """Mode-k unfolding: rows indexed by mode k, columns by the other modes (C order)."""
    return np.moveaxis(Y, k, 0).reshape(Y.shape[k], -1)


def mode_product(Y: np.ndarray, M: np.ndarray, k: int) -> np.ndarray:
    """Y x_k M, where M has shape (J, I_k): contracts mode k of Y with the columns of M."""
    Yk = np.moveaxis(Y, k, 0)
    out = np.tensordot(M, Yk, axes=([1], [0]))
    return np.moveaxis(out, 0, k)


def fix_signs(U: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of every column positive (first index on ties)."""
    U = U.copy()
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return U


def st_hosvd(T: np.ndarray, ranks):
    """Returns (core, [W1, W2, W3], [sigma_1, sigma_2, sigma_3]) with W_k of shape (I_k, r_k).

    sigma_k holds all singular values of the mode-k unfolding seen at step k.
    """
    Y = np.asarray(T, dtype=np.float64)
    factors, sigmas = [], []
    for k in range(Y.ndim):
        Uk, s, _ = np.linalg.svd(unfold(Y, k), full_matrices=False)
        Wk = fix_signs(Uk[:, : ranks[k]])
        factors.append(Wk)
        sigmas.append(s)
        Y = mode_product(Y, Wk.T, k)
    return Y, factors, sigmas


def tucker_full(core: np.ndarray, factors) -> np.ndarray:
    """core x_1 W1 x_2 W2 x_3 W3."""
    Y = core
    for k, W in enumerate(factors):
        Y = mode_product(Y, W, k)
    return Y


def ranks_for_precision(T: np.ndarray, eps: float):
    """Smallest r_k per mode with sum_{i > r_k} sigma_i^2 <= eps^2 ||T||_F^2 / d (ST-HOSVD
    truncation rule giving ||T - T~||_F <= eps ||T||_F), computed sequentially."""
    Y = np.asarray(T, dtype=np.float64)
    d = Y.ndim
    thr = eps * eps * float((Y * Y).sum()) / d
    ranks = []
    for k in range(d):
        Uk, s, _ = np.linalg.svd(unfold(Y, k), full_matrices=False)
        tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1][1:], [0.0]])
        r = int(np.argmax(tail <= thr)) + 1
        ranks.append(r)
        Y = mode_product(Y, fix_signs(Uk[:, :r]).T, k)
    return tuple(ranks)
