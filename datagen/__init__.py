"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random inputs: scattered points in a box and the values of a
smooth synthetic field at those points.  It holds none of the compression method's
arithmetic (no basis, no interpolation, no decomposition, no least squares), so the
oracle and the HIP path can both consume it without sharing method code.

The fields stand in for the paper's combustion data (Section 6), which is not
available: 3-D scattered points carrying smooth multi-scale structure (a sum of
Gaussian bumps plus a sinusoid), optional measurement noise and, for the corrector
workload, one sharp tanh front.

Random streams come from ``numpy.random.SeedSequence(seed).spawn(8)``:
0 points, 1 field parameters, 2 noise, 3 front plane, 4 held-out points,
5 per-variable parameters (batched workload), 6 extra points.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

STREAM_POINTS, STREAM_FIELD, STREAM_NOISE, STREAM_FRONT, STREAM_HELDOUT, STREAM_VARS, STREAM_EXTRA = range(7)


def _streams(seed: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(8)]


@dataclass
class FieldParams:
    """Parameters of one synthetic field, defined on reference coordinates in [-1,1]^3."""
    centers: np.ndarray          # (G, d) in [-0.8, 0.8]
    widths: np.ndarray           # (G,)  in (0.1, 0.4)
    amps: np.ndarray             # (G,)  N(0, 1)
    sin_amp: float = 0.3
    front_normal: Optional[np.ndarray] = None   # (3,) unit vector, or None
    front_offset: float = 0.0
    front_width: float = 0.02

    def __call__(self, xi: np.ndarray) -> np.ndarray:
        """Field value at reference coordinates ``xi`` of shape (n, d), d = 3 or 4 (the centres
        have d columns), in float64."""
        xi = np.asarray(xi, dtype=np.float64)
        out = self.sin_amp * np.sin(3.0 * xi[:, 0]) * np.cos(2.0 * xi[:, 1]) * np.sin(xi[:, 2])
        if xi.shape[1] == 4:
            out = out * np.cos(1.5 * xi[:, 3])
        for c, w, a in zip(self.centers, self.widths, self.amps):
            d2 = ((xi - c) ** 2).sum(axis=1)
            out += a * np.exp(-d2 / (2.0 * w * w))
        if self.front_normal is not None:
            out += np.tanh((xi @ self.front_normal - self.front_offset) / self.front_width)
        return out


def draw_field(rng: np.random.Generator, n_gauss: int, front: bool = False,
               front_rng: Optional[np.random.Generator] = None, d: int = 3) -> FieldParams:
    centers = rng.uniform(-0.8, 0.8, size=(n_gauss, d))
    widths = rng.uniform(0.1, 0.4, size=n_gauss)
    amps = rng.standard_normal(n_gauss)
    fp = FieldParams(centers=centers, widths=widths, amps=amps)
    if front:
        fr = front_rng if front_rng is not None else rng
        nrm = fr.standard_normal(3)
        fp.front_normal = nrm / np.linalg.norm(nrm)
        fp.front_offset = float(fr.uniform(-0.5, 0.5))
    return fp


def uniform_points(rng: np.random.Generator, n: int, lo, hi) -> np.ndarray:
    """(n, d) float64 points, d = len(lo), i.i.d. uniform in the box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n, lo.shape[0]))


def to_reference(pts: np.ndarray, lo, hi) -> np.ndarray:
    """Affine map of box coordinates onto [-1,1]^d (used only to evaluate the synthetic field)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return 2.0 * (np.asarray(pts, np.float64) - lo) / (hi - lo) - 1.0


@dataclass
class Workload:
    """One seeded problem instance: points, values and the method parameters it is run with."""
    name: str
    seed: int
    lo: tuple
    hi: tuple
    pts: np.ndarray               # (N, d), dtype = dtype
    vals: np.ndarray              # (N,),   dtype = dtype
    grid: tuple
    rank: tuple
    degree: tuple
    interp_fraction: float
    n_samples: int
    dtype: type = np.float64
    fieldp: Optional[FieldParams] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pts.shape[0])

    def soa(self):
        """Contiguous coordinate arrays, one per mode, then the values (structure of arrays)."""
        p = self.pts
        return tuple(np.ascontiguousarray(p[:, k]) for k in range(p.shape[1])) + (
            np.ascontiguousarray(self.vals),)


def make_workload(name: str, seed: int, n: int, n_gauss: int, grid, rank, degree,
                  interp_fraction: float, n_samples: int, dtype=np.float64,
                  noise_std: float = 0.0, front: bool = False,
                  lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)) -> Workload:
    st = _streams(seed)
    pts = uniform_points(st[STREAM_POINTS], n, lo, hi)
    fp = draw_field(st[STREAM_FIELD], n_gauss, front=front, front_rng=st[STREAM_FRONT], d=len(lo))
    # Values are computed from the points as they will be stored (rounded to dtype first),
    # so that a float32 workload's values are the field at its float32 points.
    pts = pts.astype(dtype)
    vals = fp(to_reference(pts.astype(np.float64), lo, hi))
    if noise_std > 0:
        vals = vals + noise_std * st[STREAM_NOISE].standard_normal(n)
    vals = vals.astype(dtype)
    return Workload(name=name, seed=seed, lo=tuple(lo), hi=tuple(hi), pts=pts, vals=vals,
                    grid=tuple(grid), rank=tuple(rank), degree=tuple(degree),
                    interp_fraction=interp_fraction, n_samples=n_samples, dtype=dtype, fieldp=fp)


# ---------------------------------------------------------------------------------------
# Named workloads.  Sizes follow the workload table of the build (small FP64 parity case,
# FP32 case at scale, its mixed-precision form, the batched form and the corrector form).
# ---------------------------------------------------------------------------------------

def small_f64(n: int = 20_000, n_samples: int = 2_000) -> Workload:
    """20k points in [-1,1]^3, 6 Gaussians + sinusoid, 10% -> 32^3 grid, ranks 8^3, degree 15."""
    return make_workload("small_f64", seed=1, n=n, n_gauss=6, grid=(32, 32, 32), rank=(8, 8, 8),
                         degree=(15, 15, 15), interp_fraction=0.10, n_samples=n_samples,
                         dtype=np.float64)


def large_f32(n: int = 2_000_000, n_samples: int = 200_000, grid=(128, 128, 128),
              rank=(24, 24, 24), degree=(31, 31, 31)) -> Workload:
    """2M points, 40 Gaussians + sinusoid + N(0,1e-3) noise, 5% -> 128^3, ranks 24^3, degree 31."""
    return make_workload("large_f32", seed=2, n=n, n_gauss=40, grid=grid, rank=rank,
                         degree=degree, interp_fraction=0.05, n_samples=n_samples,
                         dtype=np.float32, noise_std=1e-3)


def spacetime_f32(n: int = 2_000_000, n_samples: int = 52_000, rank=(12, 12, 12, 12),
                  degree=(31, 31, 31, 31), grid=(32, 32, 32, 32)) -> Workload:
    """A 4-way (space plus time) field standing in for the paper's space-time data (Sec. 6):
    2M points in [-1,1]^3 x [0,1], 40 Gaussians in four dimensions times a sinusoid, N(0,1e-3)
    noise, ranks 12^4 (R = 20,736) and degree 31; M = 52,000 rows is about 2.5 R."""
    return make_workload("spacetime_f32", seed=6, n=n, n_gauss=40, grid=grid, rank=rank,
                         degree=degree, interp_fraction=0.05, n_samples=n_samples,
                         dtype=np.float32, noise_std=1e-3, lo=(-1.0, -1.0, -1.0, 0.0),
                         hi=(1.0, 1.0, 1.0, 1.0))


def corrector_field(n: int = 600_000) -> Workload:
    """Large-case field plus a sharp tanh front of width 0.02 along a random plane."""
    return make_workload("corrector", seed=5, n=n, n_gauss=40, grid=(128, 128, 128),
                         rank=(24, 24, 24), degree=(31, 31, 31), interp_fraction=0.05,
                         n_samples=200_000, dtype=np.float32, noise_std=1e-3, front=True)


@dataclass
class BatchedWorkload:
    """Many field variables on one shared point set (anisotropic box [0,4]x[0,1]x[0,1])."""
    seed: int
    lo: tuple
    hi: tuple
    pts: np.ndarray                       # (N, 3) float32
    vals: list                            # V arrays (N,) float32
    ranks: list                           # V tuples (r1, r2, r3)
    degrees: list                         # V ints
    grid: tuple
    interp_fraction: float
    n_samples: int


def batched(n_vars: int = 48, n: int = 4_000_000, sample_fraction: float = 0.05,
            grid=(128, 128, 128), rmin: int = 4, rmax: int = 32, pmin: int = 15, pmax: int = 31,
            n_gauss: int = 6) -> BatchedWorkload:
    lo, hi = (0.0, 0.0, 0.0), (4.0, 1.0, 1.0)
    st = _streams(4)
    pts = uniform_points(st[STREAM_POINTS], n, lo, hi).astype(np.float32)
    xi = to_reference(pts.astype(np.float64), lo, hi)
    fields, ranks, degrees = [], [], []
    for vseed in np.random.SeedSequence(4).spawn(n_vars):
        rng = np.random.default_rng(vseed)
        # A (ranks, degree) draw is usable only if every r_k is at most the product of the
        # other two ranks (a Tucker rank condition) and at most p + 1 (r_k factor functions
        # in a space of dimension p + 1 would be linearly dependent); otherwise redraw.
        while True:
            r = tuple(int(x) for x in rng.integers(rmin, rmax + 1, size=3))
            p = int(rng.integers(pmin, pmax + 1))
            if all(r[k] <= r[(k + 1) % 3] * r[(k + 2) % 3] and r[k] <= p + 1 for k in range(3)):
                break
        fields.append(draw_field(rng, n_gauss))
        ranks.append(r)
        degrees.append(p)
    # the field values are independent per variable: evaluate them on a few threads
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        vals = list(ex.map(lambda fp: fp(xi).astype(np.float32), fields))
    return BatchedWorkload(seed=4, lo=lo, hi=hi, pts=pts, vals=vals, ranks=ranks,
                           degrees=degrees, grid=tuple(grid), interp_fraction=0.05,
                           n_samples=int(round(sample_fraction * n)))


def points_only(seed: int, n: int, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0),
                dtype=np.float32, stream: int = STREAM_EXTRA) -> np.ndarray:
    """Extra evaluation points (for example decompression targets), uniform in the box."""
    st = _streams(seed)
    return uniform_points(st[stream], n, lo, hi).astype(dtype)


def random_model_parts(seed: int, rank, degree, density: float = 0.6, scale: float = 1.0):
    """A random functional-Tucker model: core (r1, .., rd) and per-mode coefficient matrices
    (n_k, r_k) with a random sparsity pattern.  Used where a test needs a model that does
    not come from a fit (for example to plant a field that lies exactly in the model span)."""
    rng = np.random.default_rng(seed)
    core = scale * rng.standard_normal(tuple(rank))
    coefs = []
    for k in range(len(rank)):
        n_k = degree[k] + 1
        c = rng.standard_normal((n_k, rank[k])) / np.sqrt(n_k)
        mask = rng.random((n_k, rank[k])) < density
        mask[0, :] = True          # keep every column non-zero
        coefs.append(np.where(mask, c, 0.0))
    return core, coefs
