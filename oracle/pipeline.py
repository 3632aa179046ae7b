"""Algorithm 1 (compression) followed by Algorithm 2 (core re-estimation) — oracle.

Test infrastructure only.  Each stage calls the oracle module that restates the
corresponding part of the paper.
"""
from __future__ import annotations

import numpy as np

from .basis import to_reference
from .interp import grid_nodes, idw_to_grid
from .lsq import refit_core
from .model import Model
from .sampler import STREAM_INTERP, sample_without_replacement
from .sparsefit import fit_factor, fit_factor_choice
from .sthosvd import st_hosvd


def interpolation_subset(seed: int, n: int, fraction: float) -> np.ndarray:
    """K = round(fraction * N) indices (stream 1), sorted."""
    k = int(round(fraction * n))
    return sample_without_replacement(seed, STREAM_INTERP, n, k)


def reference_coords(pts: np.ndarray, lo, hi) -> np.ndarray:
    pts = np.asarray(pts, dtype=np.float64)
    return np.stack([to_reference(pts[:, k], lo[k], hi[k]) for k in range(len(lo))], axis=1)


def compress(pts, vals, lo, hi, grid, rank, degree, interp_fraction, seed,
             idw_k: int = 8, idw_power: float = 2.0, solver: str = "omp", wavelet=None) -> Model:
    """Algorithm 1: interpolate a random subset onto the grid, ST-HOSVD at fixed ranks,
    then a sparse Legendre fit of every singular vector.  The returned model carries the
    ST-HOSVD core alpha_0.  The number of modes d (3 or 4) is len(grid)."""
    pts = np.asarray(pts, dtype=np.float64)
    vals = np.asarray(vals, dtype=np.float64)
    sub = interpolation_subset(seed, pts.shape[0], interp_fraction)
    xi = reference_coords(pts[sub], lo, hi)
    T = idw_to_grid(xi, vals[sub], grid, k=idw_k, power=idw_power)
    core0, W, sig = st_hosvd(T, rank)
    if wavelet is None:
        coefs = [fit_factor(W[k], grid_nodes(grid[k]), degree[k], solver) for k in range(len(grid))]
        wav = ()
    else:   # wavelet = (s, q): every column chooses between P_p and W_{s,q} (Algorithm 1)
        s, q = wavelet
        coefs = [fit_factor_choice(W[k], grid_nodes(grid[k]), degree[k], s, q, solver) for k in range(len(grid))]
        wav = tuple((s, q) for _ in grid)
    return Model(tuple(lo), tuple(hi), tuple(rank), tuple(degree), core0, coefs,
                 info={"grid_tensor": T, "factors": W, "sigmas": sig, "subset": sub}, wavelet=wav)


def fit(pts, vals, lo, hi, grid, rank, degree, interp_fraction, n_samples, seed,
        idw_k: int = 8, idw_power: float = 2.0, solver: str = "omp", wavelet=None) -> Model:
    """Algorithm 1 then Algorithm 2 (uniformly sampled rows, normal equations)."""
    m = compress(pts, vals, lo, hi, grid, rank, degree, interp_fraction, seed, idw_k, idw_power, solver,
                 wavelet)
    alpha, idx, G, h = refit_core(m, np.asarray(pts, np.float64), vals, n_samples, seed)
    out = m.with_core(alpha)
    out.info.update({"core0": m.core, "ls_rows": idx})
    return out
