"""Sparse Legendre fit of each singular vector (oracle, test infrastructure).

Sec. 4.2 represents column j of W^(k), sampled at the grid nodes, as a function
w_j(y) = sum_i c_i phi_i(y) with few non-zero c_i, found by sparsity-regularised least
squares (Sec. 3, eq. (3)-(5)) with the regularisation chosen by leave-one-out error.  The
paper uses Lasso-LARS (``oracle.lars``, solver "lars"); the default solver here is
orthogonal matching pursuit, a greedy solver of the l0-constrained problem (3), with the same
leave-one-out model selection:

1. start from the residual r = z and an empty support S;
2. repeatedly add the column m not in S with the largest normalised correlation
   |Phi_m^T r| / ||Phi_m|| (lowest m on ties), refit c_S by least squares (Householder QR)
   and update r = z - Phi_S c_S;
3. after every step record the leave-one-out (PRESS) error (1/I) sum_i (r_i / (1 - h_ii))^2,
   where h_ii is the leverage of node i, the i-th diagonal entry of the hat matrix
   Phi_S (Phi_S^T Phi_S)^-1 Phi_S^T; a support that fits a node of leverage 1 exactly has an
   undefined leave-one-out error (0/0) and scores +inf;
4. stop when |S| reaches min(n, I - 2) or ||r|| <= 1e-14 ||z||;
5. keep the support size with the smallest PRESS (the smaller size on ties).
"""
from __future__ import annotations

import numpy as np

from .basis import legendre_orthonormal


def ls_qr(Phi: np.ndarray, z: np.ndarray):
    """Least-squares coefficients by Householder QR, and the thin Q factor."""
    Q, R = np.linalg.qr(Phi, mode="reduced")
    c = np.linalg.solve(R, Q.T @ z)  # R is upper triangular and non-singular here
    return c, Q


def omp_loo(Phi: np.ndarray, z: np.ndarray, tol: float = 1e-14):
    """Returns (support: int array in selection order, coefficients, press list)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    I, n = Phi.shape
    znorm = np.linalg.norm(z)
    if znorm == 0.0:
        return np.zeros(0, dtype=np.int64), np.zeros(0), []
    colnorm = np.linalg.norm(Phi, axis=0)
    support = []
    coefs = []
    press = []
    r = z.copy()
    tmax = min(n, I - 2)
    for _ in range(tmax):
        score = np.abs(Phi.T @ r) / colnorm
        score[support] = -1.0
        m = int(np.argmax(score))
        support.append(m)
        c, Q = ls_qr(Phi[:, support], z)
        r = z - Phi[:, support] @ c
        h = (Q * Q).sum(axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            loo = r / (1.0 - h)
        pr = float(np.mean(loo * loo))
        press.append(pr if pr == pr else np.inf)     # 0/0 at a node of leverage 1: undefined
        coefs.append(c)
        if np.linalg.norm(r) <= tol * znorm:
            break
    best = int(np.argmin(press))          # first minimum = smaller support on ties
    return np.asarray(support[: best + 1], dtype=np.int64), coefs[best], press


def fit_factor(W: np.ndarray, nodes: np.ndarray, p: int, solver: str = "omp") -> np.ndarray:
    """Sparse coefficient matrix C (p+1, r) with W[:, j] ~ Phi(nodes) @ C[:, j]; solver "omp"
    (this module) or "lars" (Lasso-LARS path of ``oracle.lars``), both with leave-one-out
    selection."""
    from .lars import lars_loo
    fit = {"omp": omp_loo, "lars": lars_loo}[solver]
    Phi = legendre_orthonormal(nodes, p)
    C = np.zeros((p + 1, W.shape[1]), dtype=np.float64)
    for j in range(W.shape[1]):
        S, c, _ = fit(Phi, W[:, j])
        C[S, j] = c
    return C


def fit_factor_choice(W: np.ndarray, nodes: np.ndarray, p: int, s: int, q: int,
                      solver: str = "omp") -> np.ndarray:
    """Algorithm 1 steps 5-6: every column is fitted in P_p and in the wavelet space W_{s,q}
    (``oracle.wavelets``, q <= p) with leave-one-out selection, and the fit with the smaller
    leave-one-out error is kept (P_p on ties).  Returns C over the mode basis: rows 0..p are
    phi_0..phi_p, then the (q + 1)(2^s - 1) detail functions."""
    from .lars import lars_loo
    from .wavelets import mode_basis, wavelet_columns
    if not (0 <= q <= p and s >= 1):
        raise ValueError("need s >= 1 and 0 <= q <= p")
    fit = {"omp": omp_loo, "lars": lars_loo}[solver]
    B = mode_basis(nodes, p, s, q)
    wcols = wavelet_columns(p, s, q)
    C = np.zeros((B.shape[1], W.shape[1]), dtype=np.float64)
    for j in range(W.shape[1]):
        SL, cL, prL = fit(B[:, : p + 1], W[:, j])
        SW, cW, prW = fit(B[:, wcols], W[:, j])
        if not prL and not prW:
            continue
        if not prW or (prL and min(prL) <= min(prW)):
            C[SL, j] = cL
        else:
            C[wcols[SW], j] = cW
    return C


def press_bruteforce(Phi_S: np.ndarray, z: np.ndarray) -> float:
    """Leave-one-out error by refitting without each node in turn (for pinning PRESS)."""
    I = Phi_S.shape[0]
    errs = np.empty(I)
    for i in range(I):
        keep = np.arange(I) != i
        c, *_ = np.linalg.lstsq(Phi_S[keep], z[keep], rcond=None)
        errs[i] = z[i] - Phi_S[i] @ c
    return float(np.mean(errs * errs))
