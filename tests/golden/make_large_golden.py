"""Writes the oracle's reference for the full-size FP32 workload (2M points, ranks 24^3,
degree 31, M = 200,000 sampled rows): the model of Algorithm 1 and the core of
Algorithm 2 computed in float64 by the oracle alone.

    python tests/golden/make_large_golden.py      (about 5-10 minutes on 8 cores)

Output: tests/golden/large_f32_reference.npz with
  coefs0, coefs1, coefs2   sparse Legendre coefficients (32 x 24 each)
  core0                    ST-HOSVD core (24^3)
  alpha                    FP64 core re-estimated from the M sampled rows
  h                        A^T v over the sampled rows
  gram_diag                diagonal of A^T A
  gram_rows, gram_cols,    a seeded sample of lower-triangle entries of A^T A (row >= col):
  gram_vals                  126,976 pairs uniform over the triangle, then the whole 64 x 64
                             block in the far corner (rows R-64..R-1, columns 0..63)
  eig_min, eig_max         extreme eigenvalues of A^T A
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from oracle import lsq, pipeline  # noqa: E402


def main():
    t0 = time.time()
    w = datagen.large_f32()
    pts = w.pts.astype(np.float64)
    vals = w.vals.astype(np.float64)
    m0 = pipeline.compress(pts, vals, w.lo, w.hi, w.grid, w.rank, w.degree, w.interp_fraction, w.seed)
    print(f"compress done {time.time() - t0:.1f} s, nnz {m0.nnz()}", flush=True)
    idx = lsq.sample_rows(w.seed, w.n, w.n_samples)
    G, h = lsq.normal_equations(m0, pts[idx], vals[idx], chunk=4096)
    print(f"normal equations done {time.time() - t0:.1f} s", flush=True)
    alpha = lsq.solve_cholesky(G, h)
    ev = np.linalg.eigvalsh(G)
    print(f"solve + eigenvalues done {time.time() - t0:.1f} s, kappa {ev[-1] / ev[0]:.3e}", flush=True)
    R = G.shape[0]
    rng = np.random.default_rng(20240611)
    a, b = rng.integers(0, R, 126976), rng.integers(0, R, 126976)
    rows, cols = np.maximum(a, b), np.minimum(a, b)
    fr, fc = np.meshgrid(np.arange(R - 64, R), np.arange(64), indexing="ij")
    rows = np.concatenate([rows, fr.reshape(-1)]).astype(np.int32)
    cols = np.concatenate([cols, fc.reshape(-1)]).astype(np.int32)
    np.savez_compressed(os.path.join(HERE, "large_f32_reference.npz"), coefs0=m0.coefs[0], coefs1=m0.coefs[1],
                        coefs2=m0.coefs[2], core0=m0.core, alpha=alpha, h=h, gram_diag=np.diag(G).copy(),
                        gram_rows=rows, gram_cols=cols, gram_vals=G[rows, cols],
                        eig_min=ev[0], eig_max=ev[-1])


if __name__ == "__main__":
    main()
