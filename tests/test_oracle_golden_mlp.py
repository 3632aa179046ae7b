"""Pins of the storage convention against the paper's Table 2 and of the FP64 corrector
network (finite differences and the closed form of Adam's first step)."""
import os

import numpy as np
import pytest

from oracle import mlp
from oracle.model import Model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_compression.txt")


def _rows():
    rows, cores = [], []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "CORE":
            cores.append((f[1], float(f[2]), [int(x) for x in f[3:]]))
        else:
            rows.append((f[0], float(f[1]), float(f[2]), float(f[3]), float(f[4])))
    return rows, cores


def test_table2_ratio_is_double_precision_original_over_stored_bytes():
    # Table 2 is consistent with ratio = 8 bytes x points / stored bytes (kB = 1000 B);
    # Model.compression_ratio uses exactly this convention.
    rows, _ = _rows()
    for name, n, prec, ratio, kb in rows:
        assert 8.0 * n / (kb * 1000.0) == pytest.approx(ratio, rel=0.01)
    # a model whose values occupy exactly 155 kB at SP3D's size gives the printed ratio
    R = 25 * 24 * 8
    nnz = 155_000 // 8 - R
    coefs = [np.zeros((nnz, 1)), np.zeros((1, 1)), np.zeros((1, 1))]
    coefs[0][:, 0] = 1.0
    m = Model((-1,) * 3, (1,) * 3, (25, 24, 8), (nnz - 1, 0, 0), np.zeros((25, 24, 8)), coefs)
    assert m.paper_bytes() == 8 * (R + nnz)
    assert m.compression_ratio(75_000_000) == pytest.approx(3879, rel=0.01)


def test_table1_core_sizes():
    _, cores = _rows()
    sizes = {(d, p): int(np.prod(r)) for d, p, r in cores}
    assert sizes[("SP3D", 1e-2)] == 4800          # the R of the self-convergence study
    assert sizes[("SP3D", 1e-4)] == 48450
    assert sizes[("SP4D", 1e-2)] == 62700


def test_mlp_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1)
    for k in p:
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)
    x = rng.uniform(-1, 1, (16, 3))
    t = rng.standard_normal(16)
    _, g = mlp.loss_and_grads(p, x, t)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for i in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grads(p, x, t)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grads(p, x, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert g[k].reshape(-1)[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_silu_closed_forms():
    z = np.array([-3.0, 0.0, 2.0])
    np.testing.assert_allclose(mlp.silu(z), z / (1 + np.exp(-z)))
    assert mlp.silu_grad(np.array([0.0]))[0] == 0.5


def test_adam_first_step_closed_form():
    # after one step with bias correction, m^ = g and v^ = g^2, so the update is -lr g/(|g|+eps)
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -1e-3, 0.0])}
    opt = mlp.Adam(p, lr=1e-2)
    out = opt.step(dict(p), g)
    exp = p["w"] - 1e-2 * g["w"] / (np.abs(g["w"]) + 1e-8)
    np.testing.assert_allclose(out["w"], exp, rtol=1e-13)


def test_param_count():
    assert mlp.n_params() == 3 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4481


def test_batch_indices_counter_form_and_range():
    from oracle.sampler import batch_indices, splitmix64, bounded, stream_state
    b0 = batch_indices(5, 0, 16, 1000)
    b3 = batch_indices(5, 3, 16, 1000)
    z = splitmix64(stream_state(5, 3), 64)
    np.testing.assert_array_equal(b0, bounded(z[:16], np.uint64(1000)).astype(np.int64))
    np.testing.assert_array_equal(b3, bounded(z[48:64], np.uint64(1000)).astype(np.int64))
    assert b0.min() >= 0 and b0.max() < 1000


def test_oracle_training_reduces_loss_on_a_ridge():
    rng = np.random.default_rng(4)
    xi = rng.uniform(-1, 1, (4000, 3))
    t = np.tanh((xi @ np.array([0.6, 0.8, 0.0]) - 0.1) / 0.1)
    p0 = mlp.init_params(2)
    p1, losses = mlp.train(p0, xi, t, steps=600, batch=256, seed=1, lr=3e-3)
    assert np.mean(losses[-20:]) < 0.2 * np.mean(losses[:5])
    np.testing.assert_array_equal(mlp.flatten(mlp.unflatten(mlp.flatten(p1))), mlp.flatten(p1))
