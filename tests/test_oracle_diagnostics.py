"""Diagnostics of the randomised least squares (Sec. 5; Sec. 6, the leverage histograms and the
self-convergence of the core against the sample count) on the oracle, at the shape of the 20,000
point FP64 workload (ranks 8 x 8 x 8, so R = 512; Legendre degree 15; uniform points).

The paper's figures are measured on its own data, so their values are not reproduced here
(parity unpinned for the values); what is checked is what the method guarantees:

* leverage scores sum to the rank before and after mixing (the mixing is orthogonal), and the
  mixing spreads them: before, a few rows near the box corners carry most of the leverage (the
  Legendre basis peaks at the ends of the interval); after, every mixed row is close to the
  mean R / N;
* sampling mixed rows gives a better conditioned sampled design than sampling the rows
  themselves, at every sample count;
* the self-convergence ||alpha(M + D) - alpha(M)|| / ||alpha(M + D)||, D = R / 5 (the paper's
  increment of 1,000 against R = 4,800), falls by more than an order of magnitude between
  M = 1.05 R and M = 12 R.
"""
import numpy as np
import pytest

import datagen
from oracle import lsq, mixing
from oracle.model import Model as OModel
from oracle.sampler import STREAM_LS, sample_without_replacement

R_SHAPE, DEG, SEED = (8, 8, 8), (15, 15, 15), 3
SWEEP = (1.05, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0, 6.0, 8.0, 12.0)


@pytest.fixture(scope="module")
def problem():
    wl = datagen.small_f64()
    core, coefs = datagen.random_model_parts(5, R_SHAPE, DEG)
    om = OModel(wl.lo, wl.hi, R_SHAPE, DEG, core, coefs)
    W = lsq.design_rows(lsq.factor_values(om, wl.pts))
    N = mixing.mixed_length(wl.n)
    FW, Fu, idx = mixing.mixed_problem(om, wl.pts, wl.vals, N, SEED)
    assert np.array_equal(idx, np.arange(N))        # S = N keeps every mixed row, in order
    return wl, om, W, FW, Fu


def test_leverage_spreads_after_mixing(problem):
    wl, om, W, FW, _ = problem
    R, n, N = W.shape[1], W.shape[0], FW.shape[0]
    before, after = lsq.leverage_scores(W), lsq.leverage_scores(FW)
    assert abs(before.sum() - R) <= 1e-9 * R and abs(after.sum() - R) <= 1e-9 * R
    bins = [0, 0.25, 0.5, 0.75, 1, 1.5, 2, 4, 8, np.inf]
    hb = np.histogram(before * n / R, bins)[0]
    ha = np.histogram(after * N / R, bins)[0]
    print("leverage / mean, bins", bins[1:], "\nbefore", hb, "\nafter ", ha)
    # before: coherent (max far above the mean, spread wider than the mean)
    assert before.max() >= 10 * R / n and before.std() >= before.mean()
    # after: every mixed row within 50% of the mean, spread below 10% of it
    assert after.max() <= 1.5 * R / N and after.min() >= 0.5 * R / N
    assert after.std() <= 0.1 * after.mean()


def test_mixed_samples_are_better_conditioned(problem):
    wl, om, W, FW, _ = problem
    R, n, N = W.shape[1], W.shape[0], FW.shape[0]
    # the sampled mixed problem of Algorithm 2 is the full mixed matrix at the sampled rows
    S = int(1.5 * R)
    A_s, _, idx_s = mixing.mixed_problem(om, wl.pts, wl.vals, S, SEED)
    assert np.array_equal(A_s, FW[idx_s])
    cw = np.linalg.cond(W)
    for f in SWEEP:
        M = int(f * R)
        c_plain = np.linalg.cond(W[lsq.sample_rows(SEED, n, M)])
        c_mixed = np.linalg.cond(FW[sample_without_replacement(SEED, STREAM_LS, N, M)])
        assert cw <= c_mixed < c_plain, (f, cw, c_mixed, c_plain)


def test_self_convergence_sweep(problem):
    wl, om, W, FW, Fu = problem
    R, N = W.shape[1], FW.shape[0]
    D = R // 5
    sc_plain, sc_mixed = [], []
    for f in SWEEP:
        M = int(f * R)
        a1 = lsq.refit_core(om, wl.pts, wl.vals, M, SEED)[0].reshape(-1)
        a2 = lsq.refit_core(om, wl.pts, wl.vals, M + D, SEED)[0].reshape(-1)
        sc_plain.append(np.linalg.norm(a2 - a1) / np.linalg.norm(a2))
        i1 = sample_without_replacement(SEED, STREAM_LS, N, M)
        i2 = sample_without_replacement(SEED, STREAM_LS, N, M + D)
        b1 = lsq.solve_cholesky(FW[i1].T @ FW[i1], FW[i1].T @ Fu[i1])
        b2 = lsq.solve_cholesky(FW[i2].T @ FW[i2], FW[i2].T @ Fu[i2])
        sc_mixed.append(np.linalg.norm(b2 - b1) / np.linalg.norm(b2))
    print("M / R", SWEEP, "\nplain", np.round(sc_plain, 4), "\nmixed", np.round(sc_mixed, 4))
    for sc in (sc_plain, sc_mixed):
        assert sc[0] >= 10 * sc[-1]
        assert max(sc[SWEEP.index(4.0):]) < min(sc[:SWEEP.index(1.5) + 1])
