"""Interpolation of scattered data onto an equispaced grid (oracle, test infrastructure).

Sec. 4.1: a small random subset of the data (about 10%) is interpolated onto an
equispaced grid I_1 x ... x I_d, and the grid tensor is then Tucker-decomposed.  The paper
says "linear interpolation"; this implementation interpolates by inverse distance weighting over
the k = 8 nearest subset points with power 2, which needs no triangulation of scattered
3-D data.  Readings taken:
* grid nodes are equispaced in reference coordinates and include both end points,
  eta_i = -1 + 2 i / (I - 1);
* distances are Euclidean in reference coordinates;
* a node that coincides with a data point takes that point's value exactly.
The exact k-nearest-neighbour search uses scipy's cKDTree as a library primitive.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def grid_nodes(I: int) -> np.ndarray:
    """Equispaced nodes on [-1, 1] including the end points."""
    return -1.0 + 2.0 * np.arange(I, dtype=np.float64) / (I - 1)


def grid_points(grid) -> np.ndarray:
    """All grid nodes, C order (last mode fastest), shape (I1*I2*I3, 3)."""
    axes = [grid_nodes(I) for I in grid]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def idw_weights_value(dist: np.ndarray, vals: np.ndarray, power: float) -> np.ndarray:
    """sum_i v_i d_i^-p / sum_i d_i^-p per row; an exact hit (d = 0) returns that value."""
    out = np.empty(dist.shape[0], dtype=np.float64)
    hit = dist[:, 0] == 0.0
    out[hit] = vals[hit, 0]
    d = dist[~hit]
    w = 1.0 / d ** power
    out[~hit] = (w * vals[~hit]).sum(axis=1) / w.sum(axis=1)
    return out


def idw_to_grid(xi: np.ndarray, v: np.ndarray, grid, k: int = 8, power: float = 2.0) -> np.ndarray:
    """Interpolate scattered (xi, v) onto the grid; returns a float64 tensor of shape grid.

    xi: (K, 3) reference coordinates of the subset; v: (K,) values.
    """
    xi = np.asarray(xi, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    k = min(k, xi.shape[0])
    nodes = grid_points(grid)
    tree = cKDTree(xi)
    dist, idx = tree.query(nodes, k=k)
    if k == 1:
        dist, idx = dist[:, None], idx[:, None]
    return idw_weights_value(dist, v[idx], power).reshape(tuple(grid))
