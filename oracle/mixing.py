"""Randomized mixing of the least-squares rows (Algorithm 2 steps 2-4), oracle, test
infrastructure: plain numpy in FP64, written for clarity, not speed.

Algorithm 2 flips the sign of every row of W and u at random (D), mixes the rows with a
fast transform (F) so that no row carries a large share of the information (the leverage
scores spread out), samples S rows uniformly (S) and solves the sampled least-squares
problem min || S F D W alpha - S F D u ||.

Readings taken (the paper fixes none of them):
* F is the normalised Walsh-Hadamard transform H_N / sqrt(N) in Sylvester order,
  H[i][k] = (-1)^popcount(i & k), the real orthogonal fast transform with the same mixing
  property as the FFT the paper names (the subsampled randomized Hadamard transform).  N is
  the smallest power of two >= max(n, 4096) (``mixed_length``; a floor of 4096 rows keeps
  the transform in whole blocks and changes nothing but the count of zero rows); rows
  n .. N-1 of W and u are zero before mixing.
* D: sign of row i is -1 when the top bit of output i of SplitMix64 stream 5 is set
  (stream_state(seed, 5); outputs numbered from 0 as in ``sampler``), +1 otherwise.
* S: S distinct rows of [0, N), uniformly without replacement and sorted (stream 2, as the
  unmixed sampling of ``lsq``).
* The sampled problem is solved by its normal equations with a Cholesky factorisation, as
  the unmixed one (``lsq.solve_cholesky``).
"""
from __future__ import annotations

import numpy as np

from .lsq import design_rows, factor_values, solve_cholesky
from .model import Model
from .sampler import STREAM_LS, sample_without_replacement, splitmix64, stream_state

STREAM_SIGNS = 5


def next_pow2(n: int) -> int:
    N = 1
    while N < n:
        N *= 2
    return N


def mixed_length(n: int) -> int:
    return max(4096, next_pow2(n))


def signs(seed: int, N: int) -> np.ndarray:
    """D: +-1 (float64) for rows 0 .. N-1."""
    z = splitmix64(stream_state(seed, STREAM_SIGNS), N)
    return np.where((z >> np.uint64(63)) != 0, -1.0, 1.0)


def fwht(X: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along axis 0 (length a power of two): the
    butterflies (a, b) -> (a + b, a - b) over strides 1, 2, 4, ..."""
    Y = np.array(X, dtype=np.float64, copy=True)
    N = Y.shape[0]
    h = 1
    while h < N:
        Y = Y.reshape((N // (2 * h), 2, h) + Y.shape[1:])
        a = Y[:, 0].copy()
        b = Y[:, 1].copy()
        Y[:, 0] = a + b
        Y[:, 1] = a - b
        Y = Y.reshape((N,) + Y.shape[3:])
        h *= 2
    return Y


def mixed_problem(model: Model, pts: np.ndarray, vals: np.ndarray, n_samples: int, seed: int):
    """(A, b, idx): the S sampled rows of F D W and F D u."""
    pts = np.asarray(pts, np.float64)
    vals = np.asarray(vals, np.float64)
    n = pts.shape[0]
    N = mixed_length(n)
    W = design_rows(factor_values(model, pts))
    Wp = np.zeros((N, W.shape[1]))
    Wp[:n] = W
    up = np.zeros(N)
    up[:n] = vals
    d = signs(seed, N)
    FW = fwht(d[:, None] * Wp) / np.sqrt(N)
    Fu = fwht(d * up) / np.sqrt(N)
    idx = sample_without_replacement(seed, STREAM_LS, N, n_samples)
    return FW[idx], Fu[idx], idx


def refit_core_mixed(model: Model, pts: np.ndarray, vals: np.ndarray, n_samples: int, seed: int):
    """Algorithm 2 with mixing: (alpha, G, h) of the sampled mixed problem."""
    A, b, _ = mixed_problem(model, pts, vals, n_samples, seed)
    G = A.T @ A
    h = A.T @ b
    return solve_cholesky(G, h), G, h
