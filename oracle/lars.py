"""Lasso-modified least angle regression with leave-one-out model selection (oracle, test
infrastructure): plain numpy in FP64.

Sec. 3 relaxes the sparse regression problem (3) to the Lasso (5), min ||z - Phi v||^2 +
lambda ||v||_1, and solves it with the Lasso modification of least angle regression (Efron,
Hastie, Johnstone, Tibshirani 2004), choosing the regularisation by a fast leave-one-out
error (Cawley and Talbot 2004) computed, as in Blatman and Sudret (2011), for the ordinary
least-squares refit on each active set met along the path.

The path, in the published notation (columns scaled to unit norm, X = Phi diag(1/||Phi_m||)):
* c = X^T (z - mu) are the current correlations and C = max_{j in A} |c_j|; the active set A
  starts with the column of largest |c_j|;
* with s_A = sign(c_A) and X_A = X[:, A] diag(s_A): G_A = X_A^T X_A, A_A = (1^T G_A^-1 1)^(-1/2),
  w_A = A_A G_A^-1 1, u_A = X_A w_A (the equiangular direction) and a = X^T u_A;
* the next column to enter is reached after gamma_hat = min+ over j not in A of
  (C - c_j) / (A_A - a_j) and (C + c_j) / (A_A + a_j);
* Lasso modification: coefficient j in A moves by gamma d_j, d_j = s_j w_j, and changes sign
  after gamma_j = -beta_j / d_j; if the smallest positive gamma_j comes first, the step stops
  there and that column leaves A;
* mu += gamma u_A, beta_A += gamma d_A.

Readings taken (the paper fixes none of them):
* ties for the entering column go to the lowest index; a column that has just left cannot
  re-enter in the next step (its correlation equals C at that point);
* the path stops when |A| reaches min(n, I - 2) (as the OMP path), when the correlations
  vanish (C <= 1e-14 C_0), or after the last step (all of a full-rank design active);
* every active set after an event of the path is refitted by least squares (Householder QR)
  and scored by PRESS = (1/I) sum_i (r_i / (1 - h_ii))^2; the first set with the smallest
  PRESS is kept (refit coefficients, support in path order); the path also stops once a
  refit leaves a residual ||r|| <= 1e-14 ||z||.
"""
from __future__ import annotations

import numpy as np

from .sparsefit import ls_qr


def lasso_lars_path(X: np.ndarray, z: np.ndarray, max_active: int, tol: float = 1e-14):
    """Events of the Lasso-LARS path on unit-norm columns X: a list of
    (active set in entry order, beta on X after the event, 'add' | 'drop' | 'end')."""
    X = np.asarray(X, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    I, n = X.shape
    beta = np.zeros(n)
    mu = np.zeros(I)
    c = X.T @ z
    C0 = float(np.max(np.abs(c))) if n else 0.0
    events = []
    if C0 == 0.0 or max_active < 1:
        return events
    active = [int(np.argmax(np.abs(c)))]
    events.append((tuple(active), beta.copy(), "add"))
    barred = -1
    for _ in range(64 * n):
        c = X.T @ (z - mu)
        s = np.sign(c[active])
        C = float(np.max(np.abs(c[active])))
        if C <= tol * C0:
            break
        XA = X[:, active] * s
        g1 = np.linalg.solve(XA.T @ XA, np.ones(len(active)))
        AA = 1.0 / np.sqrt(g1.sum())
        w = AA * g1
        u = XA @ w
        a = X.T @ u
        gamma_hat, j_hat = C / AA, -1          # C / A_A: every correlation reaches zero
        for j in range(n):
            if j in active or j == barred:
                continue
            for num, den in ((C - c[j], AA - a[j]), (C + c[j], AA + a[j])):
                if den != 0.0:
                    g = num / den
                    if 0.0 < g < gamma_hat:
                        gamma_hat, j_hat = g, j
        d = s * w
        gamma_til, k_til = np.inf, -1
        for idx, j in enumerate(active):
            if d[idx] != 0.0:
                g = -beta[j] / d[idx]
                if 0.0 < g < gamma_til:
                    gamma_til, k_til = g, idx
        barred = -1
        if gamma_til < gamma_hat:
            mu = mu + gamma_til * u
            beta[active] += gamma_til * d
            j_out = active.pop(k_til)
            beta[j_out] = 0.0
            barred = j_out
            events.append((tuple(active), beta.copy(), "drop"))
            continue
        mu = mu + gamma_hat * u
        beta[active] += gamma_hat * d
        if j_hat < 0:
            events.append((tuple(active), beta.copy(), "end"))
            break
        if len(active) >= max_active:
            break
        active.append(j_hat)
        events.append((tuple(active), beta.copy(), "add"))
    return events


def lars_loo(Phi: np.ndarray, z: np.ndarray, tol: float = 1e-14):
    """Returns (support in path order, least-squares coefficients on it, press list)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    I, n = Phi.shape
    znorm = np.linalg.norm(z)
    if znorm == 0.0:
        return np.zeros(0, dtype=np.int64), np.zeros(0), []
    colnorm = np.linalg.norm(Phi, axis=0)
    events = lasso_lars_path(Phi / colnorm, z, min(n, I - 2), tol)
    supports, coefs, press = [], [], []
    for A, _, _ in events:
        if not A:
            continue
        S = list(A)
        c, Q = ls_qr(Phi[:, S], z)
        r = z - Phi[:, S] @ c
        h = (Q * Q).sum(axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            loo = r / (1.0 - h)
        supports.append(S)
        coefs.append(c)
        pr = float(np.mean(loo * loo))
        press.append(pr if pr == pr else np.inf)     # 0/0 at a node of leverage 1: undefined
        if np.linalg.norm(r) <= tol * znorm:
            break
    best = int(np.argmin(press))
    return np.asarray(supports[best], dtype=np.int64), coefs[best], press
